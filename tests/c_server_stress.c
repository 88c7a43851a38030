/* Concurrency stress of the serving scheduler's host code, in plain C, on a
 * dry-run server (iqa_server_create_dry: the same scheduling, no GPU).  Two
 * threads submit requests while a third polls completions; the main thread
 * then drains and destroys the server.  Built with ThreadSanitizer (host code
 * only) by tests/test_sanitizers.py, which fails on any report.
 *
 * Exit status 0 and "stress ok" on stdout when every request completed once
 * with IQA_OK. */
#include <inttypes.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "iqa.h"

#define SUBMITTERS 2
#define PER_THREAD 4000
#define CHUNK 8

static iqa_server *sv;
static int32_t ref_ids[3];
static atomic_int stop_polling;
static atomic_long polled;
static atomic_long bad;

/* The dry run never dereferences these: aligned stand-ins for device
 * buffers. */
static const float *fake(uintptr_t a) { return (const float *)(a << 8); }

static void *submitter(void *arg) {
    const uint64_t id = (uint64_t)(uintptr_t)arg;
    iqa_request reqs[CHUNK];
    for (int i = 0; i < PER_THREAD; i += CHUNK) {
        memset(reqs, 0, sizeof(reqs));
        for (int k = 0; k < CHUNK; ++k) {
            const int n = i + k;
            reqs[k].snapshot_dev = fake(1 + (uintptr_t)(n % 5));
            reqs[k].lisi = (float *)fake(100 + (uintptr_t)n);
            reqs[k].auglisi = (float *)fake(200000 + (uintptr_t)n);
            reqs[k].NT = (n % 2) ? 32 : 64;
            reqs[k].ref_id = ref_ids[n % 3];
            reqs[k].tag = id * 1000000u + (uint64_t)n;
        }
        if (iqa_server_submit(sv, reqs, CHUNK) != IQA_OK) atomic_fetch_add(&bad, 1);
    }
    return NULL;
}

static void take(iqa_completion *buf, int64_t cap) {
    const int64_t n = iqa_server_poll(sv, buf, cap);
    for (int64_t i = 0; i < n; ++i)
        if (buf[i].status != IQA_OK) atomic_fetch_add(&bad, 1);
    atomic_fetch_add(&polled, (long)n);
}

static void *poller(void *arg) {
    (void)arg;
    iqa_completion buf[256];
    while (!atomic_load(&stop_polling)) take(buf, 256);
    return NULL;
}

int main(void) {
    iqa_server_opts o;
    memset(&o, 0, sizeof(o));
    o.hbm_budget_bytes = (int64_t)1 << 30;
    o.streams = 4;
    o.max_batch = 64;
    o.D = 5e-7f;
    o.C1 = o.C2 = o.C = 1e-6f;
    o.idle_spin_ns = 100000;
    /* a batch of b bytes "completes" 2 us + b / (4000 B/ns) after its launch */
    if (iqa_server_create_dry(&o, 2000, 4000.0, &sv) != IQA_OK) return 2;
    const int64_t Ns[3] = {512, 1024, 2048};
    for (int r = 0; r < 3; ++r)
        if (iqa_server_add_reference(sv, fake(1000 + (uintptr_t)r), Ns[r], &ref_ids[r]) != IQA_OK)
            return 3;
    pthread_t sub[SUBMITTERS], pol;
    pthread_create(&pol, NULL, poller, NULL);
    for (int t = 0; t < SUBMITTERS; ++t)
        pthread_create(&sub[t], NULL, submitter, (void *)(uintptr_t)(t + 1));
    for (int t = 0; t < SUBMITTERS; ++t) pthread_join(sub[t], NULL);
    const iqa_status d = iqa_server_drain(sv, 120000);
    atomic_store(&stop_polling, 1);
    pthread_join(pol, NULL);
    iqa_completion buf[256];
    for (int k = 0; k < 1000 && atomic_load(&polled) < (long)SUBMITTERS * PER_THREAD; ++k)
        take(buf, 256);
    iqa_server_stats st;
    memset(&st, 0, sizeof(st));
    iqa_server_get_stats(sv, &st);
    iqa_server_destroy(sv);
    const long want = (long)SUBMITTERS * PER_THREAD;
    printf("drain %d, completed %" PRId64 " of %ld, polled %ld, batches %" PRId64 ", bad %ld\n",
           (int)d, st.completed, want, atomic_load(&polled), st.batches, atomic_load(&bad));
    if (d != IQA_OK || st.completed != want || atomic_load(&polled) != want ||
        atomic_load(&bad) != 0)
        return 1;
    printf("stress ok\n");
    return 0;
}
