// Adjoint (backward) of the Pair-HMM forward algorithm on gfx950.
//
// The paper computes only the forward likelihood (arXiv 2411.11547,
// Section II-A, Eq. 1-4).  Its derivatives follow from the same DP run
// backwards: with B_X(i,j) = dL/dX(i,j) and B(m,.) seeded by the result
// formula L = sum_j M(m,j) + I(m,j), every term of Eq. (1)-(3) sends its
// coefficient back to its source cell,
//
//   B_M(i,j) = alpha_{i+1} Bl(i+1,j+1) + delta_{i+1} B_I(i+1,j) + zeta_i B_D(i,j+1)
//   B_I(i,j) = beta_{i+1}  Bl(i+1,j+1) + eps_{i+1}  B_I(i+1,j)
//   B_D(i,j) = beta_{i+1}  Bl(i+1,j+1) + eps_i      B_D(i,j+1)
//   Bl(i,j)  = lam_ij B_M(i,j)
//
// and d log10 L / d log10 theta_i (the posterior expected number of uses of
// theta_i) is a sum over row i of forward value x coefficient x backward
// value, divided by L.
//
// Layout: the lane structure of the forward sweep (P lanes per pair, K rows
// per lane).  Memory is bounded by checkpoints:
//  * row checkpoints: every lane stores the values of the row above its
//    first row as it receives them (one row every K rows, every column);
//  * column checkpoints: every kAdjC steps each lane stores its K-row state.
// The backward walks the forward steps in reverse, kAdjC at a time: each
// lane reloads its state at the start of the block, recomputes the block's
// kAdjC columns in registers from the stored row above (no lane exchange is
// needed for that), then runs the reverse wavefront over them.  All lanes
// sit at the same forward step (each on its own column), so the block
// structure is the same in every lane.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ph_device.h"
#include "ph_internal.h"

namespace ph {

__constant__ double c_prob[256];  // Phred q -> 10^(-q/10), computed on the host in FP64

hipError_t upload_luts_adjoint()
{
    double t[256];
    for (int q = 0; q < 256; ++q) t[q] = pow(10.0, -(double)q / 10.0);
    return hipMemcpyToSymbol(HIP_SYMBOL(c_prob), t, sizeof(t));
}

template <int P, int K>
struct AdjCfg {
    static constexpr int G = 64 / P;
    // E[code][row][lane] = (lam, w) with w = 1 for a mismatch, 0 otherwise
    static constexpr int CODE_BYTES = K * 512;
    static constexpr int E_BYTES = kCodes * CODE_BYTES;
};

// Per-pair prologue shared by both kernels: the pair's record, the per-row
// parameters of the lane's K rows (absorbing rows past the read end, as in
// the forward sweep), the (lam, w) table and the haplotype staged in LDS
// with PAD outside columns 1..n.
template <int P, int K>
struct AdjPair {
    using C = AdjCfg<P, K>;
    int lane, g, t, idx;
    bool valid;
    AdjRec rec;
    int64_t ro;
    int m, n, S;
    float al[K], be[K], de[K], ep[K], ze[K];
    char *E;
    const uint8_t *hs;  // staged codes; column j sits at hs[j + P]

    __device__ __forceinline__ void init(const AdjArgs &A, char *lds)
    {
        lane = threadIdx.x;
        g = lane / P;
        t = lane % P;
        const int first = blockIdx.x * C::G;
        idx = first + g;
        valid = idx < A.nrec;
        // groups past the end of the list mirror group 0 and never write
        rec = A.recs[valid ? idx : first];
        S = __builtin_amdgcn_readlane(rec.S, 0);
        const DevProblem &pb = A.pb;
        ro = pb.read_offset[rec.read];
        m = (int)(pb.read_offset[rec.read + 1] - ro);
        n = rec.n;
        E = lds;
        char *mine = E + lane * 8;
        auto slot = [&](int c, int r) -> float * { return (float *)(mine + c * C::CODE_BYTES + r * 512); };
#pragma unroll 1
        for (int r = 0; r < K; ++r) {
            const int i = t * K + r;
            const int ic = min(i, m - 1);
            const RowPar p = load_row(pb, A.lin_params, ro + ic, c_prob);
            const bool real = i < m;
            *slot(0, r) = real ? (float)p.a : 0.f;
            *slot(1, r) = real ? (float)p.b : 0.f;
            *slot(2, r) = real ? (float)p.d : (i == m ? 1.f : 0.f);
            *slot(3, r) = real ? (float)p.e : 1.f;
            *slot(4, r) = real ? (float)p.z : 0.f;
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
                float2 v = make_float2(0.f, 0.f);
                if (real && c != kPad) v = match ? make_float2((float)p.lm, 0.f) : make_float2((float)p.lx, 1.f);
                *(float2 *)(mine + c * C::CODE_BYTES + r * 512) = v;
            }
        }
        uint8_t *h = (uint8_t *)(lds + C::E_BYTES + g * A.hs_bytes);
        const uint8_t *hap = pb.hap_bases + pb.hap_offset[rec.hap];
        const int len = S + P + 2;
        for (int x = t; x < len; x += P) {
            const int j = x - P;
            h[x] = (j >= 1 && j <= n) ? (uint8_t)clamp_code(hap[j - 1]) : (uint8_t)kPad;
        }
        hs = h;
        __syncthreads();
    }

    __device__ __forceinline__ const char *ecol(int s) const
    {
        return E + (int)hs[s - t + 1 + P] * C::CODE_BYTES + lane * 8;
    }
};

// One forward step of the lane's K rows in the plain formulation of
// Eq. (1)-(3) (D kept unscaled, as the gradients need it): (mo, io, do_)
// hold column j-1 on entry, (mn, in, dn) receive column j; (mu, iu) and
// (md, id, dd) are the row above at columns j and j-1.
template <int K>
__device__ __forceinline__ void adj_cell_step(const float (&mo)[K], const float (&io)[K], const float (&do_)[K],
                                              float (&mn)[K], float (&in)[K], float (&dn)[K], float mu,
                                              float iu, float md, float id, float dd, const float *lam,
                                              const float (&al)[K], const float (&be)[K],
                                              const float (&de)[K], const float (&ep)[K],
                                              const float (&ze)[K])
{
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const float x = fma(al[r], md, be[r] * (id + dd));
        const float mr = lam[r] * x;
        const float ir = fma(ep[r], iu, de[r] * mu);
        const float dr = fma(ep[r], do_[r], ze[r] * mo[r]);
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

// Checkpointed forward: also writes the row above every lane at every step
// (slot s+1 = step s, slot 0 = the initial diagonal) and every lane's state
// before steps 0, kAdjC, 2 kAdjC, ...  Workspace of a group at ws + ws_off:
// [S+1][3][P] row checkpoints, then [S/kAdjC][3][K][P] column checkpoints.
template <int P, int K>
__global__ __launch_bounds__(64) void k_adj_fwd(AdjArgs A)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    AdjPair<P, K> pr;
    pr.init(A, lds);
    const int t = pr.t, S = pr.S;
    const bool wr = pr.valid;
    float *bnd = A.ws + pr.rec.ws_off;
    float *ck = bnd + (int64_t)(S + 1) * 3 * P;
    const float edge = (t == 0) ? (float)(ldexp(1.0, 120) / (double)pr.n) : 0.f;  // D(0, j) = 1/n, scaled

    float M[K], I[K], D[K];
#pragma unroll
    for (int r = 0; r < K; ++r) M[r] = I[r] = D[r] = 0.f;
    float md = 0.f, id = 0.f, dd = edge;
    if (wr) {
        bnd[0 * P + t] = 0.f;
        bnd[1 * P + t] = 0.f;
        bnd[2 * P + t] = dd;
    }
    double acc = 0.0;
    for (int s0 = 0; s0 < S; s0 += kAdjC) {
        if (wr) {
            float *cq = ck + (int64_t)(s0 / kAdjC) * 3 * K * P + t;
#pragma unroll
            for (int r = 0; r < K; ++r) {
                cq[(0 * K + r) * P] = M[r];
                cq[(1 * K + r) * P] = I[r];
                cq[(2 * K + r) * P] = D[r];
            }
        }
#pragma unroll
        for (int c = 0; c < kAdjC; ++c) {
            const int s = s0 + c;
            const float mu = shift_up<P>(M[K - 1]);
            const float iu = shift_up<P>(I[K - 1]);
            const float du = shift_up<P>(D[K - 1]) + edge;
            if (wr) {
                float *b = bnd + (int64_t)(s + 1) * 3 * P + t;
                b[0] = mu;
                b[P] = iu;
                b[2 * P] = du;
            }
            float lam[K];
            const char *e = pr.ecol(s);
#pragma unroll
            for (int r = 0; r < K; ++r) lam[r] = *(const float *)(e + r * 512);
            adj_cell_step<K>(M, I, D, M, I, D, mu, iu, md, id, dd, lam, pr.al, pr.be, pr.de, pr.ep, pr.ze);
            md = mu;
            id = iu;
            dd = du;
            acc += (double)I[K - 1];
        }
    }
    if (wr && t == P - 1) A.Ls[pr.idx] = acc;
}

template <int P, int K>
__device__ __forceinline__ void adj_load_block(const float *bnd, const float *ck, int q, int t, float (&cq)[3][K],
                                               float (&bq)[kAdjC + 1][3])
{
    const float *c0 = ck + (int64_t)q * 3 * K * P + t;
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int r = 0; r < K; ++r) cq[v][r] = c0[(v * K + r) * P];
    const float *b0 = bnd + (int64_t)q * kAdjC * 3 * P + t;
#pragma unroll
    for (int c = 0; c <= kAdjC; ++c)
#pragma unroll
        for (int v = 0; v < 3; ++v) bq[c][v] = b0[(c * 3 + v) * P];
}

// Backward: reverse wavefront over the checkpointed forward, gradients of
// u_p log10 L_p added into the per-read-base gradient array.
template <int P, int K>
__global__ __launch_bounds__(64) void k_adj_bwd(AdjArgs A)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    AdjPair<P, K> pr;
    pr.init(A, lds);
    const int t = pr.t, S = pr.S;
    const float *bnd = A.ws + pr.rec.ws_off;
    const float *ck = bnd + (int64_t)(S + 1) * 3 * P;

    // parameters of the row below the lane's last row: the next lane's first
    // row, or below the group a virtual row that only passes B_I up
    const float an_x = shift_down<P>(pr.al[0]);
    const float bn_x = shift_down<P>(pr.be[0]);
    const float dn_x = shift_down<P>(pr.de[0]);
    const float en_x = shift_down<P>(pr.ep[0]) + ((t == P - 1) ? 1.f : 0.f);

    // B is seeded with 2^SB, SB chosen so that forward x backward products
    // sit near 2^30 whatever L is
    const double Ls = A.Ls[pr.idx < A.nrec ? pr.idx : blockIdx.x * AdjCfg<P, K>::G];
    const bool good = (Ls >= A.threshold) && (Ls <= 3.0e38);
    const int SB = good ? 30 - ilogb(Ls) : 0;
    const float bscale = good ? ldexpf(1.f, SB) : 0.f;
    const float edge_bi = (t == P - 1) ? bscale : 0.f;

    float BI[K], BD[K], BL[K];
    float Aa[K], Ab[K], Am[K], Ad[K], Aei[K], Aed[K], Az[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
        BI[r] = BD[r] = BL[r] = 0.f;
        Aa[r] = Ab[r] = Am[r] = Ad[r] = Aei[r] = Aed[r] = Az[r] = 0.f;
    }
    float bl_dn_prev = 0.f;

    const int Q = S / kAdjC;
    float cn[3][K], bn[kAdjC + 1][3];
    adj_load_block<P, K>(bnd, ck, Q - 1, t, cn, bn);
    for (int q = Q - 1; q >= 0; --q) {
        float F[kAdjC + 1][3][K];
        float bb[kAdjC + 1][3];
#pragma unroll
        for (int v = 0; v < 3; ++v)
#pragma unroll
            for (int r = 0; r < K; ++r) F[0][v][r] = cn[v][r];
#pragma unroll
        for (int c = 0; c <= kAdjC; ++c)
#pragma unroll
            for (int v = 0; v < 3; ++v) bb[c][v] = bn[c][v];
        if (q > 0) adj_load_block<P, K>(bnd, ck, q - 1, t, cn, bn);

        // recompute the block's columns from the lane's checkpoint
#pragma unroll
        for (int c = 0; c < kAdjC; ++c) {
            float lam[K];
            const char *e = pr.ecol(q * kAdjC + c);
#pragma unroll
            for (int r = 0; r < K; ++r) lam[r] = *(const float *)(e + r * 512);
            adj_cell_step<K>(F[c][0], F[c][1], F[c][2], F[c + 1][0], F[c + 1][1], F[c + 1][2], bb[c + 1][0],
                             bb[c + 1][1], bb[c][0], bb[c][1], bb[c][2], lam, pr.al, pr.be, pr.de, pr.ep,
                             pr.ze);
        }

        // reverse wavefront over the block
#pragma unroll
        for (int c = kAdjC - 1; c >= 0; --c) {
            const char *e = pr.ecol(q * kAdjC + c);
            float lam[K], w[K];
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const float2 v = *(const float2 *)(e + r * 512);
                lam[r] = v.x;
                w[r] = v.y;
            }
            const float bi_dn = shift_down<P>(BI[0]) + edge_bi;
            const float bl_dn = shift_down<P>(BL[0]);
            float bid = bi_dn;          // B_I of the row below, this column
            float bl_below = bl_dn_prev; // Bl of the row below, next column
#pragma unroll
            for (int r = K - 1; r >= 0; --r) {
                const float bld = bl_below;
                const float an = (r == K - 1) ? an_x : pr.al[r + 1];
                const float bnr = (r == K - 1) ? bn_x : pr.be[r + 1];
                const float dn = (r == K - 1) ? dn_x : pr.de[r + 1];
                const float en = (r == K - 1) ? en_x : pr.ep[r + 1];
                const float tb = bnr * bld;
                const float bi = fma(en, bid, tb);
                const float bd = fma(pr.ep[r], BD[r], tb);
                const float bm = fma(an, bld, fma(dn, bid, pr.ze[r] * BD[r]));
                const float bl = lam[r] * bm;
                // forward values around (i, j): row above at j and j-1, own row at j-1 and j
                const float mu = (r == 0) ? bb[c + 1][0] : F[c + 1][0][r - 1];
                const float iu = (r == 0) ? bb[c + 1][1] : F[c + 1][1][r - 1];
                const float mdg = (r == 0) ? bb[c][0] : F[c][0][r - 1];
                const float idg = (r == 0) ? bb[c][1] : F[c][1][r - 1];
                const float ddg = (r == 0) ? bb[c][2] : F[c][2][r - 1];
                Aa[r] = fma(mdg, bl, Aa[r]);
                Ab[r] = fma(idg + ddg, bl, Ab[r]);
                Am[r] = fma(w[r] * F[c + 1][0][r], bm, Am[r]);
                Ad[r] = fma(mu, bi, Ad[r]);
                Aei[r] = fma(iu, bi, Aei[r]);
                Aed[r] = fma(F[c][2][r], bd, Aed[r]);
                Az[r] = fma(F[c][0][r], bd, Az[r]);
                bl_below = BL[r];  // still the next column's value: row r-1's diagonal
                BI[r] = bi;
                BD[r] = bd;
                BL[r] = bl;
                bid = bi;
            }
            bl_dn_prev = bl_dn;
        }
    }

    // expected uses per row: g = coefficient x sum / (L_s 2^SB), times the
    // upstream gradient of the pair; lam_match by sum over the row's M entries
    if (!pr.valid) return;
    const double u = A.grad_in[pr.rec.out];
    if (u == 0.0) return;  // contributes nothing, even where the FP32 sweep underflowed
    const double inv = good ? 1.0 / ldexp(Ls, SB) : (double)NAN;
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const int i = t * K + r;
        if (i >= pr.m) continue;
        const double ga = pr.al[r] * (double)Aa[r] * inv;
        const double gb = pr.be[r] * (double)Ab[r] * inv;
        const double gx = (double)Am[r] * inv;
        float *o = A.grad_out + (pr.ro + i) * 7;
        atomicAdd(o + 0, (float)(u * ga));
        atomicAdd(o + 1, (float)(u * gb));
        atomicAdd(o + 2, (float)(u * pr.de[r] * (double)Ad[r] * inv));
        atomicAdd(o + 3, (float)(u * pr.ep[r] * ((double)Aei[r] + (double)Aed[r]) * inv));
        atomicAdd(o + 4, (float)(u * pr.ze[r] * (double)Az[r] * inv));
        atomicAdd(o + 5, (float)(u * (ga + gb - gx)));
        atomicAdd(o + 6, (float)(u * gx));
    }
}

__global__ __launch_bounds__(256) void k_zero_f32(float *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0.f;
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
    (void)P;
    return kCodes * K * 512;
}

hipError_t launch_adj(const AdjArgs &a, int P, int K, int tiles, bool backward, hipStream_t s)
{
    const size_t lds = (size_t)kCodes * K * 512 + (size_t)(64 / P) * a.hs_bytes;
#define PH_LA(p, k)                                                                                 \
    if (P == p && K == k) {                                                                         \
        if (backward)                                                                               \
            hipLaunchKernelGGL((k_adj_bwd<p, k>), dim3(tiles), dim3(64), lds, s, a);                \
        else                                                                                        \
            hipLaunchKernelGGL((k_adj_fwd<p, k>), dim3(tiles), dim3(64), lds, s, a);                \
        return hipGetLastError();                                                                   \
    }
    PH_ADJ_CONFIGS(PH_LA)
#undef PH_LA
    return hipErrorInvalidValue;
}

hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t s)
{
    int64_t g = (n + 1023) / 1024;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_zero_f32, dim3((int)g), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace ph
