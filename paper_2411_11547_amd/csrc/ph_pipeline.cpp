// Host-input streaming forward: the workflow of arXiv 2411.11547 Section
// III-A.  The batches are cut into subsets of whole batches (stage 1); each
// subset's bases and qualities are copied to the GPU (stages 2 and 5) while
// the previous subset is binned and computed (stages 3 and 4, one plan per
// subset), and each subset's scores are copied back as soon as it finishes
// (stage 7, per subset here so that the copies overlap the next subset's
// compute).
//
// Streams: H2D copies on `h2d`, plans on `comp[k % 2]`, D2H copies on
// `d2h`.  Two compute streams let the start of subset k+1 (binning and the
// first bins' sweeps) overlap the tail of subset k (44.3 -> 41.4 ms per call
// on the mixed batch in 9 subsets).  Subsets of up to 6e10 cells by default:
// with haplotype chains, whose tiles are longer, the mixed batch runs in 4
// subsets at 36.4-36.9 ms per call against 39.1-39.4 in 9.  When every subset's inputs and outputs
// together take at most a
// quarter of the free device memory (or the caller asks for as many buffer
// sets as there are subsets), each subset gets its own buffer set and
// the copies never wait for compute: all H2D copies are issued up front and
// run back to back on the copy engine while the subsets compute.  Otherwise
// N buffer sets (2 by default) are reused in turn, and events order their
// reuse: the H2D of subset k+N waits until the compute of subset k has read
// its inputs, and the compute of subset k+N waits until the D2H of subset k
// has read its outputs.  (A copy that waits for a compute
// event is released only when the kernels queued ahead of it on the shared
// hardware queues drain, so with two sets the H2D of a subset cannot start
// before the previous subset's sweeps end.)
//
// This file is a client of the public plan API plus the HIP runtime.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "ph.h"

namespace ph {
void set_last_error(const char *msg);  // ph_api.cpp: the message of ph_last_error()
}

#ifndef PH_PIPE_COMP_STREAMS
#define PH_PIPE_COMP_STREAMS 2
#endif

namespace {

constexpr int kCompStreams = PH_PIPE_COMP_STREAMS;  // subsets alternate between these
constexpr int64_t kDefaultSubsetCells = 60000000000LL;  // cells per subset unless given

ph_status pfail(ph_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ph::set_last_error(buf);
    return st;
}

#define PCHK(x)                                                                                   \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess) return pfail(PH_ERR_HIP, "%s: %s", #x, hipGetErrorString(e_));      \
    } while (0)

// One subset: a contiguous range of batches, its rebased shape (host and
// device copies) and its plan.
struct Subset {
    int32_t b0, b1;         // batches
    int32_t r0, r1, h0, h1; // reads, haplotypes
    int64_t rb0, rb1;       // read bases
    int64_t hb0, hb1;       // haplotype bases
    int64_t out0, pairs;    // output range
    int64_t cells;
    std::vector<int32_t> bra, bha;
    std::vector<int64_t> ro, ho;
    int32_t *d_bra = nullptr, *d_bha = nullptr;
    int64_t *d_ro = nullptr, *d_ho = nullptr;
    ph_plan *plan = nullptr;
};

struct BufSet {
    uint8_t *rb = nullptr, *bq = nullptr, *iq = nullptr, *dq = nullptr, *gq = nullptr, *hb = nullptr;
    double *out = nullptr;
    uint8_t *status = nullptr;
    hipEvent_t h2d_done = nullptr, comp_done = nullptr, d2h_done = nullptr;
    bool used = false;
};

}  // namespace

struct ph_pipeline {
    int32_t nb = 0, nr = 0, nh = 0;
    int64_t P = 0, cells = 0;
    std::vector<Subset> subsets;
    int64_t max_rbases = 0, max_hbases = 0, max_pairs = 0;
    std::vector<BufSet> sets;
    hipStream_t h2d = nullptr, comp[kCompStreams] = {}, d2h = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    bool timed = false;
};

namespace {

void destroy(ph_pipeline *q)
{
    if (!q) return;
    for (auto &s : q->subsets) {
        if (s.plan) ph_plan_destroy(s.plan);
        void *bufs[] = {s.d_bra, s.d_bha, s.d_ro, s.d_ho};
        for (void *b : bufs)
            if (b) (void)hipFree(b);
    }
    for (auto &b : q->sets) {
        void *bufs[] = {b.rb, b.bq, b.iq, b.dq, b.gq, b.hb, b.out, b.status};
        for (void *x : bufs)
            if (x) (void)hipFree(x);
        hipEvent_t evs[] = {b.h2d_done, b.comp_done, b.d2h_done};
        for (auto e : evs)
            if (e) (void)hipEventDestroy(e);
    }
    hipStream_t ss[] = {q->h2d, q->d2h};
    for (auto s : ss)
        if (s) (void)hipStreamDestroy(s);
    for (auto s : q->comp)
        if (s) (void)hipStreamDestroy(s);
    if (q->t0) (void)hipEventDestroy(q->t0);
    if (q->t1) (void)hipEventDestroy(q->t1);
    delete q;
}

template <typename T>
ph_status palloc(T **p, int64_t count)
{
    const size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc((void **)p, bytes);
    if (e != hipSuccess) return pfail(PH_ERR_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    return PH_OK;
}

}  // namespace

extern "C" {

void ph_pipeline_opts_default(ph_pipeline_opts *o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->max_subset_cells = 0;
    ph_plan_opts_default(&o->plan);
}

ph_status ph_pipeline_create(const ph_shape *shape, const ph_pipeline_opts *opts_in, ph_pipeline **out)
{
    ph::set_last_error("");
    if (!shape || !out) return pfail(PH_ERR_INVALID, "shape or out is NULL");
    *out = nullptr;
    ph_pipeline_opts opts;
    if (opts_in) opts = *opts_in; else ph_pipeline_opts_default(&opts);
    const int64_t cap = opts.max_subset_cells > 0 ? opts.max_subset_cells : kDefaultSubsetCells;
    const int32_t nb = shape->num_batches, nr = shape->num_reads, nh = shape->num_haps;
    if (nb < 0 || nr < 0 || nh < 0) return pfail(PH_ERR_INVALID, "negative counts");
    if ((nb > 0 && (!shape->batch_read_begin || !shape->batch_hap_begin)) || !shape->read_offset ||
        !shape->hap_offset)
        return pfail(PH_ERR_INVALID, "shape arrays are NULL");
    const int32_t *rb = shape->batch_read_begin, *hb = shape->batch_hap_begin;
    const int64_t *ro = shape->read_offset, *ho = shape->hap_offset;
    if (nb > 0 && (rb[0] != 0 || hb[0] != 0)) return pfail(PH_ERR_INVALID, "batch ranges must start at 0");
    for (int32_t b = 0; b < nb; ++b)
        if (rb[b + 1] < rb[b] || hb[b + 1] < hb[b] || rb[b + 1] > nr || hb[b + 1] > nh)
            return pfail(PH_ERR_INVALID, "batch %d has a bad read or haplotype range", b);

    ph_pipeline *q = new ph_pipeline;
    q->nb = nb;
    q->nr = nr;
    q->nh = nh;

    // stage 1: greedy cut into subsets of whole batches, at most `cap` cells
    // each (a larger batch forms a subset of its own)
    int64_t out0 = 0;
    int32_t b = 0;
    while (b < nb) {
        Subset s{};
        s.b0 = b;
        s.out0 = out0;
        while (b < nb) {
            int64_t nsum = 0;
            for (int32_t h = hb[b]; h < hb[b + 1]; ++h) nsum += ho[h + 1] - ho[h];
            int64_t c = 0, pairs = (int64_t)(rb[b + 1] - rb[b]) * (hb[b + 1] - hb[b]);
            for (int32_t r = rb[b]; r < rb[b + 1]; ++r) c += (ro[r + 1] - ro[r]) * nsum;
            if (b > s.b0 && s.cells + c > cap) break;
            s.cells += c;
            s.pairs += pairs;
            ++b;
        }
        s.b1 = b;
        out0 += s.pairs;
        q->subsets.push_back(std::move(s));
    }
    q->P = out0;

    ph_status st = PH_OK;
    for (auto &s : q->subsets) {
        q->cells += s.cells;
        s.r0 = rb[s.b0];
        s.r1 = rb[s.b1];
        s.h0 = hb[s.b0];
        s.h1 = hb[s.b1];
        s.rb0 = ro[s.r0];
        s.rb1 = ro[s.r1];
        s.hb0 = ho[s.h0];
        s.hb1 = ho[s.h1];
        const int32_t snb = s.b1 - s.b0, snr = s.r1 - s.r0, snh = s.h1 - s.h0;
        s.bra.resize(snb + 1);
        s.bha.resize(snb + 1);
        for (int32_t i = 0; i <= snb; ++i) {
            s.bra[i] = rb[s.b0 + i] - s.r0;
            s.bha[i] = hb[s.b0 + i] - s.h0;
        }
        s.ro.resize(snr + 1);
        s.ho.resize(snh + 1);
        for (int32_t i = 0; i <= snr; ++i) s.ro[i] = ro[s.r0 + i] - s.rb0;
        for (int32_t i = 0; i <= snh; ++i) s.ho[i] = ho[s.h0 + i] - s.hb0;
        ph_shape sh{snb, s.bra.data(), s.bha.data(), snr, s.ro.data(), snh, s.ho.data()};
        st = ph_plan_create(&sh, &opts.plan, &s.plan);
        if (st != PH_OK) {  // the plan's message stays in ph_last_error()
            destroy(q);
            return st;
        }
        if ((st = palloc(&s.d_bra, snb + 1)) || (st = palloc(&s.d_bha, snb + 1)) ||
            (st = palloc(&s.d_ro, snr + 1)) || (st = palloc(&s.d_ho, snh + 1))) {
            destroy(q);
            return st;
        }
        hipError_t e = hipSuccess;
        if (e == hipSuccess) e = hipMemcpy(s.d_bra, s.bra.data(), (snb + 1) * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s.d_bha, s.bha.data(), (snb + 1) * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s.d_ro, s.ro.data(), (snr + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s.d_ho, s.ho.data(), (snh + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            destroy(q);
            return pfail(PH_ERR_HIP, "hipMemcpy: %s", hipGetErrorString(e));
        }
        q->max_rbases = std::max(q->max_rbases, s.rb1 - s.rb0);
        q->max_hbases = std::max(q->max_hbases, s.hb1 - s.hb0);
        q->max_pairs = std::max(q->max_pairs, s.pairs);
    }
    // one buffer set per subset when they all fit well inside the free
    // device memory, else two that alternate
    int64_t all_bytes = 0;
    for (const auto &s : q->subsets) all_bytes += 5 * (s.rb1 - s.rb0) + (s.hb1 - s.hb0) + 9 * s.pairs;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
    const int nsub = (int)q->subsets.size();
    int nsets = (nsub > 2 && all_bytes <= (int64_t)(free_b / 4)) ? nsub : 2;
    if (opts.buffer_sets > 0) nsets = std::max(2, opts.buffer_sets);
    nsets = std::min(nsets, nsub);
    q->sets.resize(std::max(nsets, 1));
    for (int k = 0; k < nsets; ++k) {
        BufSet &bs = q->sets[k];
        if ((st = palloc(&bs.rb, q->max_rbases)) || (st = palloc(&bs.bq, q->max_rbases)) ||
            (st = palloc(&bs.iq, q->max_rbases)) || (st = palloc(&bs.dq, q->max_rbases)) ||
            (st = palloc(&bs.gq, q->max_rbases)) || (st = palloc(&bs.hb, q->max_hbases)) ||
            (st = palloc(&bs.out, q->max_pairs)) || (st = palloc(&bs.status, q->max_pairs))) {
            destroy(q);
            return st;
        }
        hipError_t e = hipSuccess;
        if (e == hipSuccess) e = hipEventCreateWithFlags(&bs.h2d_done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&bs.comp_done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&bs.d2h_done, hipEventDisableTiming);
        if (e != hipSuccess) {
            destroy(q);
            return pfail(PH_ERR_HIP, "hipEventCreate: %s", hipGetErrorString(e));
        }
    }
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&q->h2d, hipStreamNonBlocking);
    for (auto &c : q->comp)
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&c, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&q->d2h, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&q->t0);
    if (e == hipSuccess) e = hipEventCreate(&q->t1);
    if (e != hipSuccess) {
        destroy(q);
        return pfail(PH_ERR_HIP, "stream/event creation: %s", hipGetErrorString(e));
    }
    *out = q;
    return PH_OK;
}

ph_status ph_pipeline_info(const ph_pipeline *q, int32_t *num_subsets, int64_t *num_pairs, int64_t *num_cells)
{
    ph::set_last_error("");
    if (!q) return pfail(PH_ERR_INVALID, "pipeline is NULL");
    if (num_subsets) *num_subsets = (int32_t)q->subsets.size();
    if (num_pairs) *num_pairs = q->P;
    if (num_cells) *num_cells = q->cells;
    return PH_OK;
}

ph_status ph_pipeline_forward(ph_pipeline *q, const ph_problem *hp, double *out_log10L, uint8_t *out_status)
{
    ph::set_last_error("");
    if (!q) return pfail(PH_ERR_INVALID, "pipeline is NULL");
    if (!hp) return pfail(PH_ERR_INVALID, "problem is NULL");
    if (hp->num_batches != q->nb || hp->num_reads != q->nr || hp->num_haps != q->nh)
        return pfail(PH_ERR_PLAN_MISMATCH, "problem counts differ from the pipeline's shape");
    if (q->P == 0) return PH_OK;
    if (!out_log10L || !hp->read_bases || !hp->base_qual || !hp->ins_qual || !hp->del_qual || !hp->gcp_qual ||
        !hp->hap_bases)
        return pfail(PH_ERR_INVALID, "a host array is NULL");
    PCHK(hipEventRecord(q->t0, q->h2d));
    const size_t nsub = q->subsets.size(), nsets = q->sets.size();
    // stages 2 and 5: inputs of subset k, once subset k - nsets has read them
    auto h2d = [&](size_t k) -> ph_status {
        const Subset &s = q->subsets[k];
        BufSet &bs = q->sets[k % nsets];
        const int64_t nrb = s.rb1 - s.rb0, nhb = s.hb1 - s.hb0;
        if (bs.used) PCHK(hipStreamWaitEvent(q->h2d, bs.comp_done, 0));
        PCHK(hipMemcpyAsync(bs.rb, hp->read_bases + s.rb0, nrb, hipMemcpyHostToDevice, q->h2d));
        PCHK(hipMemcpyAsync(bs.bq, hp->base_qual + s.rb0, nrb, hipMemcpyHostToDevice, q->h2d));
        PCHK(hipMemcpyAsync(bs.iq, hp->ins_qual + s.rb0, nrb, hipMemcpyHostToDevice, q->h2d));
        PCHK(hipMemcpyAsync(bs.dq, hp->del_qual + s.rb0, nrb, hipMemcpyHostToDevice, q->h2d));
        PCHK(hipMemcpyAsync(bs.gq, hp->gcp_qual + s.rb0, nrb, hipMemcpyHostToDevice, q->h2d));
        PCHK(hipMemcpyAsync(bs.hb, hp->hap_bases + s.hb0, nhb, hipMemcpyHostToDevice, q->h2d));
        PCHK(hipEventRecord(bs.h2d_done, q->h2d));
        return PH_OK;
    };
    // stages 3 and 4: binning and sweeps of subset k, once its inputs are in
    // and subset k - nsets's scores have left the output buffers; stage 7,
    // per subset: its scores back to the host
    auto compute = [&](size_t k) -> ph_status {
        Subset &s = q->subsets[k];
        BufSet &bs = q->sets[k % nsets];
        hipStream_t comp = q->comp[k % kCompStreams];
        PCHK(hipStreamWaitEvent(comp, bs.h2d_done, 0));
        if (bs.used) PCHK(hipStreamWaitEvent(comp, bs.d2h_done, 0));
        ph_problem dp{s.b1 - s.b0, s.d_bra, s.d_bha, s.r1 - s.r0, s.d_ro, bs.rb, bs.bq, bs.iq, bs.dq, bs.gq,
                      s.h1 - s.h0, s.d_ho, bs.hb};
        ph_status st = ph_forward_batch(s.plan, &dp, nullptr, bs.out, bs.status, comp);
        if (st != PH_OK) return st;
        PCHK(hipEventRecord(bs.comp_done, comp));
        PCHK(hipStreamWaitEvent(q->d2h, bs.comp_done, 0));
        PCHK(hipMemcpyAsync(out_log10L + s.out0, bs.out, s.pairs * sizeof(double), hipMemcpyDeviceToHost, q->d2h));
        if (out_status)
            PCHK(hipMemcpyAsync(out_status + s.out0, bs.status, s.pairs, hipMemcpyDeviceToHost, q->d2h));
        PCHK(hipEventRecord(bs.d2h_done, q->d2h));
        bs.used = true;
        return PH_OK;
    };
    ph_status st = PH_OK;
    if (nsets == nsub) {
        // a buffer set per subset: every H2D copy first, then the computes
        for (size_t k = 0; k < nsub && st == PH_OK; ++k) st = h2d(k);
        for (size_t k = 0; k < nsub && st == PH_OK; ++k) st = compute(k);
    } else {
        for (size_t k = 0; k < nsub && st == PH_OK; ++k) {
            st = h2d(k);
            if (st == PH_OK) st = compute(k);
        }
    }
    if (st != PH_OK) return st;
    PCHK(hipEventRecord(q->t1, q->d2h));
    PCHK(hipEventSynchronize(q->t1));
    for (auto &bs : q->sets) bs.used = false;
    q->timed = true;
    return PH_OK;
}

ph_status ph_pipeline_ms(ph_pipeline *q, float *ms)
{
    ph::set_last_error("");
    if (!q || !ms) return pfail(PH_ERR_INVALID, "pipeline or ms is NULL");
    if (!q->timed) return pfail(PH_ERR_STATE, "no ph_pipeline_forward call recorded");
    PCHK(hipEventElapsedTime(ms, q->t0, q->t1));
    return PH_OK;
}

void ph_pipeline_destroy(ph_pipeline *q) { destroy(q); }

void *ph_host_alloc(size_t bytes)
{
    void *p = nullptr;
    if (hipHostMalloc(&p, bytes ? bytes : 1, hipHostMallocDefault) != hipSuccess) return nullptr;
    return p;
}

void ph_host_free(void *p)
{
    if (p) (void)hipHostFree(p);
}

}  // extern "C"
