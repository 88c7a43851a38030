/* Compiled by tests/test_abi.py with a plain C compiler against include/iqa.h
 * and linked to libiqa_hip.so: the boundary is usable from C.  It only calls
 * entry points that return before touching a GPU. */
#include <stdio.h>
#include <string.h>

#include "iqa.h"

int main(void) {
    int fails = 0;
    iqa_launch_cfg cfg;
    const float *fake = (const float *)(unsigned long)(1u << 20);
    if (iqa_default_cfg(2048, 64, fake, fake, &cfg) != IQA_OK || cfg.vec != 4) fails |= 1;
    if (iqa_check_cfg(2048, 64, &cfg) != IQA_OK) fails |= 2;
    if (iqa_tiles(NULL, fake, 2048, 64, 5e-7f, 1e-6f, 1e-6f, 1e-6f, (float *)fake, NULL, NULL,
                  NULL) != IQA_ERR_NULL) fails |= 4;
    if (iqa_tiles(fake, fake, 2048, 63, 5e-7f, 1e-6f, 1e-6f, 1e-6f, (float *)fake, NULL, NULL,
                  NULL) != IQA_ERR_SHAPE) fails |= 8;
    if (lisi_tiles(fake, fake, 2048, 64, 5e-7f, 0.0f, 1e-6f, (float *)fake, NULL) != IQA_ERR_PARAM)
        fails |= 16;
    if (strncmp(iqa_status_str(IQA_ERR_ALIGN), "IQA_ERR_ALIGN", 13) != 0) fails |= 32;
    if (iqa_version() < 100) fails |= 64;
    /* struct sizes, compared by the test with the Python binding's mirrors */
    printf("sizes %zu %zu %zu %zu %zu %zu\n", sizeof(iqa_launch_cfg), sizeof(iqa_pair),
           sizeof(iqa_server_opts), sizeof(iqa_request), sizeof(iqa_completion),
           sizeof(iqa_server_stats));
    printf("c_abi_check %s (%d)\n", fails ? "FAILED" : "ok", fails);
    return fails;
}
