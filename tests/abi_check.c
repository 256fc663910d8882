/* A C program built against include/ffd.h and linked with libffd.so: the
 * sizes and field offsets of the public structs, and one plan of a
 * planning-only context (no GPU) through the C ABI, printed as JSON lines
 * for tests/test_abi_c.py to compare with the Python binding. */
#include <stddef.h>
#include <stdio.h>
#include <stdlib.h>

#include "ffd.h"

#define FIELD(T, f) printf("{\"struct\": \"%s\", \"field\": \"%s\", \"offset\": %zu, \"size\": %zu}\n", #T, #f, \
                           offsetof(T, f), sizeof(((T *)0)->f))
#define SIZE(T) printf("{\"struct\": \"%s\", \"sizeof\": %zu}\n", #T, sizeof(T))

int main(void) {
  SIZE(ffd_plan_summary);
  FIELD(ffd_plan_summary, link_elems);
  FIELD(ffd_plan_summary, stream_steps);
  FIELD(ffd_plan_summary, jobs);
  FIELD(ffd_plan_summary, pipelined);
  FIELD(ffd_plan_summary, per_lane);
  SIZE(ffd_plan_job);
  FIELD(ffd_plan_job, row_sel);
  FIELD(ffd_plan_job, band_count);
  FIELD(ffd_plan_job, flag_out);
  SIZE(ffd_launch_info);
  FIELD(ffd_launch_info, pipelined);
  FIELD(ffd_launch_info, helper_waves);
  FIELD(ffd_launch_info, stream_steps);
  FIELD(ffd_launch_info, per_lane);
  SIZE(ffd_tuning);
  FIELD(ffd_tuning, tried);
  SIZE(ffd_search_info);
  SIZE(ffd_server_stats);
  FIELD(ffd_server_stats, p50_ms);
  FIELD(ffd_server_stats, requests_per_launch);
  FIELD(ffd_server_stats, launches_by_rows);
  FIELD(ffd_server_stats, canceled);
  FIELD(ffd_server_stats, expired);

  /* a planning-only context: 256 compute units, 160 KiB of LDS per block */
  ffd_ctx *ctx = NULL;
  int rc = ffd_create_planner(256, 160 * 1024, &ctx);
  if (rc != FFD_OK) {
    printf("{\"error\": \"ffd_create_planner\", \"status\": %d}\n", rc);
    return 1;
  }
  /* 40 pairs of lengths 100 + 37 k and 2000 - 41 k */
  int64_t p_off[41], q_off[41];
  p_off[0] = q_off[0] = 0;
  for (int k = 0; k < 40; ++k) {
    p_off[k + 1] = p_off[k] + 100 + 37 * k;
    q_off[k + 1] = q_off[k] + 2000 - 41 * k;
  }
  ffd_plan_summary sm;
  int32_t *wave_jobs = NULL;
  ffd_plan_job *jobs = NULL;
  rc = ffd_plan_describe(ctx, FFD_OP_BATCH, p_off, 40, q_off, 40, 2, 0, 0, FFD_EUCLIDEAN, &sm, NULL, 0, NULL, 0);
  if (rc != FFD_OK && rc != FFD_E_NOMEM) {
    printf("{\"error\": \"ffd_plan_describe\", \"status\": %d, \"detail\": \"%s\"}\n", rc, ffd_last_error(ctx));
    return 1;
  }
  jobs = (ffd_plan_job *)malloc(sizeof(ffd_plan_job) * (size_t)sm.jobs);
  wave_jobs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(sm.waves + 1));
  rc = ffd_plan_describe(ctx, FFD_OP_BATCH, p_off, 40, q_off, 40, 2, 0, 0, FFD_EUCLIDEAN, &sm, jobs, sm.jobs,
                         wave_jobs, sm.waves + 1);
  if (rc != FFD_OK) {
    printf("{\"error\": \"ffd_plan_describe\", \"status\": %d}\n", rc);
    return 1;
  }
  printf("{\"plan\": {\"rows_per_lane\": %d, \"waves\": %d, \"waves_per_block\": %d, \"cooperative\": %d, "
         "\"rings\": %d, \"flags\": %d, \"link_elems\": %lld, \"stream_steps\": %lld, \"jobs\": %lld, "
         "\"pipelined\": %d, \"last_wave_jobs\": %d}}\n",
         sm.rows_per_lane, sm.waves, sm.waves_per_block, sm.cooperative, sm.rings, sm.flags,
         (long long)sm.link_elems, (long long)sm.stream_steps, (long long)sm.jobs, sm.pipelined,
         wave_jobs[sm.waves]);
  /* status codes and their text */
  printf("{\"strerror\": \"%s\"}\n", ffd_strerror(FFD_E_NOMEM));
  rc = ffd_set_tuning(ctx, 3, 0);
  printf("{\"bad_tuning_status\": %d}\n", rc);
  /* kernel timing: a planning-only context launches nothing to time */
  double ms = -1;
  int64_t launches = -1;
  int rc_on = ffd_set_kernel_timing(ctx, 1);
  rc = ffd_kernel_time(ctx, &ms, &launches);
  printf("{\"timing_on_status\": %d, \"kernel_time_status\": %d, \"ms\": %.1f, \"launches\": %lld}\n", rc_on, rc,
         ms, (long long)launches);
  free(jobs);
  free(wave_jobs);
  ffd_destroy(ctx);
  return 0;
}
