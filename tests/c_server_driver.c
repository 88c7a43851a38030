/* Drives the serving ABI from plain C, with no Python and no torch: one
 * resident reference, a set of device snapshots, one request per snapshot,
 * then drain, poll and a bitwise comparison of every served result with the
 * single-pair launch of the same geometry (iqa_serve_cfg + iqa_tiles_cfg).
 * Test infrastructure, built by the build step with a C compiler and run by
 * tests/test_gpu_c_driver.py.
 *
 *   c_server_driver IN OUT
 *
 * IN  holds int64 N, int64 NT, int64 count, then the reference and `count`
 *     snapshots (N*N float32 each, row-major).
 * OUT receives int32 [server_create, add_reference, submit, drain, polled,
 *     statuses_ok, served_equals_single], then the served LISI and augLISI
 *     matrices of every request (ns*ns float32 each, request order).
 *
 * C1 = C2 = C = 1e-6f and D = C1 / 2. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "iqa.h"

#define HIP_OK(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));     \
            exit(3);                                                              \
        }                                                                         \
    } while (0)

static void *read_all(const char *path, size_t *len) {
    FILE *f = fopen(path, "rb");
    if (!f) return NULL;
    fseek(f, 0, SEEK_END);
    long n = ftell(f);
    fseek(f, 0, SEEK_SET);
    void *buf = malloc((size_t)n);
    if (buf && fread(buf, 1, (size_t)n, f) != (size_t)n) {
        free(buf);
        buf = NULL;
    }
    fclose(f);
    *len = (size_t)n;
    return buf;
}

int main(int argc, char **argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: %s IN OUT\n", argv[0]);
        return 2;
    }
    size_t len = 0;
    char *in = read_all(argv[1], &len);
    if (!in || len < 24) {
        fprintf(stderr, "cannot read %s\n", argv[1]);
        return 2;
    }
    int64_t N, NT, count;
    memcpy(&N, in, 8);
    memcpy(&NT, in + 8, 8);
    memcpy(&count, in + 16, 8);
    const size_t npix = (size_t)N * (size_t)N;
    if (N <= 0 || NT <= 0 || N % NT != 0 || count < 1 || count > 1024 ||
        len != 24 + 4 * npix * (size_t)(count + 1)) {
        fprintf(stderr, "bad input header\n");
        return 2;
    }
    const size_t nt = (size_t)(N / NT) * (size_t)(N / NT);
    const float c = 1e-6f, d = c / 2.0f;
    const float *host = (const float *)(in + 24);

    float *ref, *snaps, *lisi, *aug, *lisi1, *aug1;
    HIP_OK(hipMalloc((void **)&ref, npix * 4));
    HIP_OK(hipMalloc((void **)&snaps, npix * 4 * (size_t)count));
    HIP_OK(hipMalloc((void **)&lisi, nt * 4 * (size_t)count));
    HIP_OK(hipMalloc((void **)&aug, nt * 4 * (size_t)count));
    HIP_OK(hipMalloc((void **)&lisi1, nt * 4 * (size_t)count));
    HIP_OK(hipMalloc((void **)&aug1, nt * 4 * (size_t)count));
    HIP_OK(hipMemcpy(ref, host, npix * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(snaps, host + npix, npix * 4 * (size_t)count, hipMemcpyHostToDevice));

    int32_t st[7] = {0, 0, 0, 0, 0, 0, 0};
    iqa_server_opts opts;
    memset(&opts, 0, sizeof(opts));
    opts.hbm_budget_bytes = (int64_t)1 << 30;
    opts.streams = 2;
    opts.max_batch = 64;
    opts.D = d;
    opts.C1 = opts.C2 = opts.C = c;
    iqa_server *sv = NULL;
    st[0] = iqa_server_create(&opts, &sv);
    int32_t rid = -1;
    if (st[0] == IQA_OK) st[1] = iqa_server_add_reference(sv, ref, N, &rid);

    iqa_request *reqs = calloc((size_t)count, sizeof(iqa_request));
    for (int64_t i = 0; i < count; ++i) {
        reqs[i].snapshot_dev = snaps + (size_t)i * npix;
        reqs[i].lisi = lisi + (size_t)i * nt;
        reqs[i].auglisi = aug + (size_t)i * nt;
        reqs[i].NT = NT;
        reqs[i].ref_id = rid;
        reqs[i].tag = (uint64_t)(1000 + i);
    }
    if (st[0] == IQA_OK && st[1] == IQA_OK) {
        st[2] = iqa_server_submit(sv, reqs, count);
        st[3] = iqa_server_drain(sv, 30000);
        iqa_completion *comps = calloc((size_t)count, sizeof(iqa_completion));
        int64_t got = 0;
        while (got < count) {
            const int64_t n = iqa_server_poll(sv, comps + got, count - got);
            if (n <= 0) break;
            got += n;
        }
        st[4] = (int32_t)got;
        int ok = got == count;
        for (int64_t i = 0; i < got; ++i)
            ok = ok && comps[i].status == IQA_OK && comps[i].tag >= 1000 &&
                 comps[i].tag < (uint64_t)(1000 + count);
        st[5] = ok;
        free(comps);
    }
    if (sv) iqa_server_destroy(sv);

    /* The same pairs as single launches with the server's geometry. */
    iqa_launch_cfg cfg;
    int same = iqa_serve_cfg(N, NT, &cfg) == IQA_OK;
    for (int64_t i = 0; same && i < count; ++i)
        same = iqa_tiles_cfg(snaps + (size_t)i * npix, ref, N, NT, d, c, c, c,
                             lisi1 + (size_t)i * nt, aug1 + (size_t)i * nt, NULL, &cfg,
                             NULL) == IQA_OK;
    HIP_OK(hipDeviceSynchronize());
    const size_t nb = nt * 4 * (size_t)count;
    float *h = malloc(nb * 4);
    HIP_OK(hipMemcpy(h, lisi, nb, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy((char *)h + nb, aug, nb, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy((char *)h + 2 * nb, lisi1, nb, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy((char *)h + 3 * nb, aug1, nb, hipMemcpyDeviceToHost));
    st[6] = same && memcmp(h, (char *)h + 2 * nb, 2 * nb) == 0;

    FILE *f = fopen(argv[2], "wb");
    if (!f) return 2;
    fwrite(st, 4, 7, f);
    fwrite(h, 1, 2 * nb, f);
    fclose(f);
    printf("c_server_driver N=%lld NT=%lld requests=%lld statuses %d %d %d %d polled %d ok %d "
           "served==single %d\n", (long long)N, (long long)NT, (long long)count, st[0], st[1],
           st[2], st[3], st[4], st[5], st[6]);

    hipFree(ref);
    hipFree(snaps);
    hipFree(lisi);
    hipFree(aug);
    hipFree(lisi1);
    hipFree(aug1);
    free(h);
    free(reqs);
    free(in);
    return 0;
}
