/* Drives the library from plain C, with no Python and no torch: device
 * memory from hipMalloc, a stream from hipStreamCreate, and the C entry points
 * of include/iqa.h.  Test infrastructure, built by the build step with a C
 * compiler and run by tests/test_gpu_c_driver.py.
 *
 *   c_gpu_driver IN OUT
 *
 * IN  holds int64 N, int64 NT, then x and y (N*N float32 each, row-major).
 * OUT receives int32 statuses [fused, lisi_tiles, auglisi_tiles, bad_align],
 * int32 fused_equals_separate, then the fused LISI, augLISI (ns*ns float32
 * each) and sums (ns*ns*4 float32), ns = N / NT.
 *
 * Every call uses C1 = C2 = C = 1e-6f and D = C1 / 2.  The last status is an
 * explicit float4 launch shape on an image offset by one float, which the
 * library must refuse with IQA_ERR_ALIGN before launching anything. */
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
    if (!in || len < 16) {
        fprintf(stderr, "cannot read %s\n", argv[1]);
        return 2;
    }
    int64_t N, NT;
    memcpy(&N, in, 8);
    memcpy(&NT, in + 8, 8);
    if (N <= 0 || NT <= 0 || N % NT != 0 || len != 16 + 8 * (size_t)N * (size_t)N) {
        fprintf(stderr, "bad input header\n");
        return 2;
    }
    const size_t npix = (size_t)N * (size_t)N;
    const size_t nt = (size_t)(N / NT) * (size_t)(N / NT);
    const float c = 1e-6f, d = c / 2.0f;

    float *x, *y, *lisi, *aug, *sums, *lisi2, *aug2, *shifted;
    HIP_OK(hipMalloc((void **)&x, npix * 4));
    HIP_OK(hipMalloc((void **)&y, npix * 4));
    HIP_OK(hipMalloc((void **)&shifted, (npix + 4) * 4));
    HIP_OK(hipMalloc((void **)&lisi, nt * 4));
    HIP_OK(hipMalloc((void **)&aug, nt * 4));
    HIP_OK(hipMalloc((void **)&sums, nt * 16));
    HIP_OK(hipMalloc((void **)&lisi2, nt * 4));
    HIP_OK(hipMalloc((void **)&aug2, nt * 4));
    HIP_OK(hipMemcpy(x, in + 16, npix * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(y, in + 16 + npix * 4, npix * 4, hipMemcpyHostToDevice));
    hipStream_t s;
    HIP_OK(hipStreamCreate(&s));

    int32_t st[4];
    st[0] = iqa_tiles(x, y, N, NT, d, c, c, c, lisi, aug, sums, s);
    st[1] = lisi_tiles(x, y, N, NT, d, c, c, lisi2, s);
    st[2] = auglisi_tiles(x, y, N, NT, c, aug2, s);
    iqa_launch_cfg cfg;
    st[3] = iqa_default_cfg(N, NT, x, y, &cfg);
    if (st[3] == IQA_OK && cfg.vec == 4)
        st[3] = iqa_tiles_cfg(shifted + 1, y, N, NT, d, c, c, c, lisi2, NULL, NULL, &cfg, s);
    else
        st[3] = -1;
    HIP_OK(hipStreamSynchronize(s));

    float *h = malloc(nt * 4 * 8);
    float *hl = h, *ha = h + nt, *hs = h + 2 * nt, *hl2 = h + 6 * nt, *ha2 = h + 7 * nt;
    HIP_OK(hipMemcpy(hl, lisi, nt * 4, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(ha, aug, nt * 4, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(hs, sums, nt * 16, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(hl2, lisi2, nt * 4, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(ha2, aug2, nt * 4, hipMemcpyDeviceToHost));
    int32_t same = memcmp(hl, hl2, nt * 4) == 0 && memcmp(ha, ha2, nt * 4) == 0;

    FILE *f = fopen(argv[2], "wb");
    if (!f) return 2;
    fwrite(st, 4, 4, f);
    fwrite(&same, 4, 1, f);
    fwrite(h, 4, nt * 6, f);
    fclose(f);
    printf("c_gpu_driver N=%lld NT=%lld statuses %d %d %d %d (%s) separate==fused %d\n",
           (long long)N, (long long)NT, st[0], st[1], st[2], st[3], iqa_status_str(st[3]),
           same);

    HIP_OK(hipStreamDestroy(s));
    hipFree(x);
    hipFree(y);
    hipFree(shifted);
    hipFree(lisi);
    hipFree(aug);
    hipFree(sums);
    hipFree(lisi2);
    hipFree(aug2);
    free(h);
    free(in);
    return 0;
}
