/* Host checks of libpairhmm's C ABI, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host code (no GPU needed): every path
 * that validates arguments and shapes before touching the device, plan and
 * pipeline creation up to the first HIP call (which fails without a GPU, so
 * the partly built plan is torn down again).  Exits 0 when every call returns the expected status. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ph.h"

static int failures = 0;

static void expect(const char *what, ph_status got, ph_status want)
{
    if (got != want) {
        fprintf(stderr, "FAIL %s: status %d, expected %d (%s)\n", what, (int)got, (int)want, ph_last_error());
        ++failures;
    }
}

static void expect_one_of(const char *what, ph_status got, ph_status a, ph_status b)
{
    if (got != a && got != b) {
        fprintf(stderr, "FAIL %s: status %d (%s)\n", what, (int)got, ph_last_error());
        ++failures;
    }
}

int main(void)
{
    /* two batches: 2 reads x 2 haplotypes, 1 read x 1 haplotype */
    int32_t rb[3] = {0, 2, 3}, hb[3] = {0, 2, 3};
    int64_t ro[4] = {0, 10, 25, 40}, ho[4] = {0, 30, 50, 51};
    ph_shape s = {2, rb, hb, 3, ro, 3, ho};
    ph_plan_opts o;
    ph_plan_opts_default(&o);
    ph_plan *plan = NULL;

    expect("NULL shape", ph_plan_create(NULL, &o, &plan), PH_ERR_INVALID);
    expect("NULL out", ph_plan_create(&s, &o, NULL), PH_ERR_INVALID);

    int64_t ro_bad[4] = {0, 10, 10, 40}; /* empty read */
    ph_shape sb = s;
    sb.read_offset = ro_bad;
    expect("empty read", ph_plan_create(&sb, &o, &plan), PH_ERR_INVALID);

    int64_t ho_bad[4] = {0, 30, 30, 51}; /* empty haplotype */
    sb = s;
    sb.hap_offset = ho_bad;
    expect("empty haplotype", ph_plan_create(&sb, &o, &plan), PH_ERR_INVALID);

    int32_t rb_bad[3] = {0, 3, 2}; /* decreasing range */
    sb = s;
    sb.batch_read_begin = rb_bad;
    expect("bad batch range", ph_plan_create(&sb, &o, &plan), PH_ERR_INVALID);

    int64_t ro_long[4] = {0, 10, 25, 25 + 65536};
    sb = s;
    sb.read_offset = ro_long;
    expect("read too long", ph_plan_create(&sb, &o, &plan), PH_ERR_UNSUPPORTED);

    ph_plan_opts ob = o;
    ob.force_p = 12;
    expect("bad force_p", ph_plan_create(&s, &ob, &plan), PH_ERR_INVALID);

    ob = o;
    ob.tune_table_path = "/nonexistent/tune.txt";
    /* the table is read after the device query: HIP error without a GPU,
     * invalid with one; either way the partly built plan is freed */
    expect_one_of("missing tune table", ph_plan_create(&s, &ob, &plan), PH_ERR_INVALID, PH_ERR_HIP);

    /* a good shape: fails at the first HIP call without a GPU */
    ph_status st = ph_plan_create(&s, &o, &plan);
    expect_one_of("good shape", st, PH_OK, PH_ERR_HIP);
    if (st == PH_OK) ph_plan_destroy(plan);

    /* calls on a NULL plan */
    expect("forward NULL plan", ph_forward_batch(NULL, NULL, NULL, NULL, NULL, NULL), PH_ERR_INVALID);
    expect("viterbi NULL plan", ph_viterbi_batch(NULL, NULL, NULL, NULL, NULL, NULL), PH_ERR_INVALID);
    expect("backward NULL plan", ph_backward_batch(NULL, NULL, NULL, NULL, NULL, NULL), PH_ERR_INVALID);
    expect("validate NULL plan", ph_validate(NULL, NULL, NULL), PH_ERR_INVALID);
    float ms[4];
    expect("stage_ms NULL plan", ph_plan_stage_ms(NULL, ms), PH_ERR_INVALID);
    int64_t cnt = 0;
    expect("rescued NULL plan", ph_plan_rescued(NULL, &cnt), PH_ERR_INVALID);
    expect("info NULL plan", ph_plan_info(NULL, NULL, NULL, NULL, NULL), PH_ERR_INVALID);
    ph_plan_destroy(NULL);

    /* pipeline: bad range, then a good shape (HIP error without a GPU) */
    ph_pipeline_opts po;
    ph_pipeline_opts_default(&po);
    ph_pipeline *pipe = NULL;
    sb = s;
    sb.batch_read_begin = rb_bad;
    expect("pipeline bad range", ph_pipeline_create(&sb, &po, &pipe), PH_ERR_INVALID);
    po.max_subset_cells = 100; /* every batch a subset of its own */
    st = ph_pipeline_create(&s, &po, &pipe);
    expect_one_of("pipeline good shape", st, PH_OK, PH_ERR_HIP);
    if (st == PH_OK) ph_pipeline_destroy(pipe);
    ph_pipeline_destroy(NULL);

    /* the allocation-free forward: shape checks before any device work; a
     * good shape reaches the device set-up (HIP error without a GPU) */
    ph_problem pb;
    memset(&pb, 0, sizeof(pb));
    pb.num_batches = 2;
    pb.num_reads = 3;
    pb.num_haps = 3;
    expect("noalloc NULL shape", ph_forward_batch_noalloc(NULL, &pb, NULL, NULL, NULL, NULL), PH_ERR_INVALID);
    sb = s;
    sb.read_offset = ro_bad;
    expect("noalloc empty read", ph_forward_batch_noalloc(&sb, &pb, NULL, NULL, NULL, NULL), PH_ERR_INVALID);
    int64_t ro_1024[4] = {0, 10, 25, 25 + 1024};
    sb = s;
    sb.read_offset = ro_1024;
    expect("noalloc read over 1023", ph_forward_batch_noalloc(&sb, &pb, NULL, NULL, NULL, NULL), PH_ERR_UNSUPPORTED);
    ph_problem pm = pb;
    pm.num_reads = 4;
    expect("noalloc count mismatch", ph_forward_batch_noalloc(&s, &pm, NULL, NULL, NULL, NULL), PH_ERR_PLAN_MISMATCH);
    expect("noalloc NULL output", ph_forward_batch_noalloc(&s, &pb, NULL, NULL, NULL, NULL), PH_ERR_INVALID);

    if (strstr(ph_version(), "gfx950") == NULL) {
        fprintf(stderr, "FAIL version %s\n", ph_version());
        ++failures;
    }
    printf("host checks: %d failures\n", failures);
    return failures ? 1 : 0;
}
