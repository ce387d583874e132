/*
 * A quench through the C ABI alone (no Python, no PyTorch): the caller
 * allocates the device buffer with hipMalloc, creates a lattice, runs n
 * sweeps on the null stream, measures, and prints the integer sums.
 *
 *   c_abi_quench <model> <L> <seed> <n> <beta> <D>
 *
 * Output, one line: "t B M Q counts[-1] counts[0] counts[+1] sd[0..8] Cx[1] Cy[1] n_r".
 */
#include <hip/hip_runtime_api.h>
#include <inttypes.h>
#include <stdio.h>
#include <stdlib.h>

#include "mcl.h"

static int fail(const char* what, int code)
{
    fprintf(stderr, "%s: %s (%d)\n", what, mcl_strerror(code), code);
    return 1;
}

int main(int argc, char** argv)
{
    if (argc != 7) {
        fprintf(stderr, "usage: %s model L seed n beta D\n", argv[0]);
        return 2;
    }
    const int model = atoi(argv[1]);
    const int64_t L = strtoll(argv[2], NULL, 10);
    const uint64_t seed = strtoull(argv[3], NULL, 10);
    const int64_t n = strtoll(argv[4], NULL, 10);
    const double beta = atof(argv[5]), D = atof(argv[6]);

    int64_t bytes = 0;
    int rc = mcl_query_bytes(model, L, &bytes);
    if (rc) return fail("mcl_query_bytes", rc);
    void* dev = NULL;
    if (hipMalloc(&dev, (size_t)bytes) != hipSuccess) {
        fprintf(stderr, "hipMalloc of %" PRId64 " bytes failed\n", bytes);
        return 1;
    }
    mcl_lattice* h = NULL;
    rc = lattice_init(&h, model, L, seed, MCL_INIT_RANDOM, dev, bytes, NULL);
    if (rc) return fail("lattice_init", rc);
    rc = sweep(h, n, beta, D);
    if (rc) return fail("sweep", rc);

    int32_t nr = 0;
    rc = mcl_rset(MCL_CORR_PROTOCOL, L, n, NULL, 0, &nr);
    if (rc != MCL_EBUFSZ && rc < 0) return fail("mcl_rset", rc);
    int32_t* r = (int32_t*)malloc(sizeof(int32_t) * (size_t)nr);
    int64_t* cx = (int64_t*)malloc(sizeof(int64_t) * (size_t)nr);
    int64_t* cy = (int64_t*)malloc(sizeof(int64_t) * (size_t)nr);
    int64_t* ns = (int64_t*)malloc(sizeof(int64_t) * (size_t)nr);
    mcl_measure_out out = {0};
    out.r = r;
    out.Cx = cx;
    out.Cy = cy;
    out.nsrc = ns;
    out.r_cap = nr;
    rc = measure(h, MCL_CORR_PROTOCOL, &out);
    if (rc) return fail("measure", rc);

    printf("%" PRId64 " %" PRId64 " %" PRId64 " %" PRId64 " %" PRId64 " %" PRId64 " %" PRId64, out.t, out.B, out.M,
           out.Q, out.counts[0], out.counts[1], out.counts[2]);
    for (int k = 0; k < 9; ++k) printf(" %" PRId64, out.sd[k]);
    printf(" %" PRId64 " %" PRId64 " %d\n", cx[1], cy[1], out.n_r);

    lattice_free(h);
    hipFree(dev);
    free(r);
    free(cx);
    free(cy);
    free(ns);
    return 0;
}
