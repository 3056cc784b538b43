/*
 * abi_client.c -- a plain C program that uses liblgf.so only through
 * include/lgf.h, as any C caller of the library would.
 *
 *   abi_client check
 *       argument checks that need no GPU: status codes of bad arguments,
 *       NULL handles, buffer sizes and the parameter defaults.
 *   abi_client run Lt Lz Ly Lx omega in.bin out.bin
 *       create an FP64 18-real lattice, load the canonical links
 *       double[V][4][3][3][2] from in.bin, run one full sweep (parity 0 then
 *       1) of overrelaxation with the given omega, measure F and theta
 *       (Eqs. (2), (5)), store the links to out.bin and destroy the handle;
 *       prints "F theta" on stdout.
 *
 * Exit status 0 on success; otherwise the failing call and lgf_last_error()
 * go to stderr.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lgf.h"

static int expect(const char *what, lgf_status got, lgf_status want)
{
    if (got != want) {
        fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, (int)got, (int)want, lgf_last_error());
        return 1;
    }
    return 0;
}

static int check(void)
{
    int bad = 0;
    const int odd[4] = {8, 8, 8, 7};
    const int ok[4] = {8, 8, 8, 8};
    lgf_lattice *h = (lgf_lattice *)0x1;
    bad += expect("create odd extent", lgf_create(odd, LGF_FP64_18, NULL, NULL, 0, &h), LGF_EINVAL);
    if (h != NULL) {
        fprintf(stderr, "create with bad dims left a handle\n");
        ++bad;
    }
    if (strlen(lgf_last_error()) == 0) {
        fprintf(stderr, "no error message after a failed call\n");
        ++bad;
    }
    bad += expect("create split format", lgf_create(ok, LGF_FP64_12S, NULL, NULL, 0, &h), LGF_EINVAL);
    bad += expect("create NULL out", lgf_create(ok, LGF_FP64_18, NULL, NULL, 0, NULL), LGF_EINVAL);
    bad += expect("destroy NULL", lgf_destroy(NULL), LGF_OK);
    bad += expect("sweep NULL", lgf_sweep(NULL, 2, 1.7, 0.0, 0, 0), LGF_EINVAL);
    bad += expect("measure NULL", lgf_measure(NULL, NULL, NULL), LGF_EINVAL);
    bad += expect("gauge_fix NULL", lgf_gauge_fix(NULL, NULL, NULL, NULL, 0), LGF_EINVAL);
    bad += expect("fix_chunk NULL", lgf_fix_chunk(NULL, 20, 1.7, 0.0, 0, 0, 1, NULL, NULL, NULL), LGF_EINVAL);
    if (lgf_required_bytes(ok, LGF_FP64_18) != (size_t)8 * 8 * 8 * 8 * 4 * 144 ||
        lgf_required_bytes(odd, LGF_FP64_18) != 0) {
        fprintf(stderr, "lgf_required_bytes\n");
        ++bad;
    }
    lgf_fix_params p;
    bad += expect("fix_params_default", lgf_fix_params_default(&p), LGF_OK);
    if (p.omega != 1.7 || p.check_every != 20 || p.max_sweeps != 100000 || p.theta_target != 1e-14) {
        fprintf(stderr, "unexpected defaults\n");
        ++bad;
    }
    if (!lgf_version() || !lgf_version()[0]) {
        fprintf(stderr, "no version string\n");
        ++bad;
    }
    if (bad == 0) printf("check ok\n");
    return bad ? 1 : 0;
}

static int run(int argc, char **argv)
{
    if (argc != 9) {
        fprintf(stderr, "usage: abi_client run Lt Lz Ly Lx omega in.bin out.bin\n");
        return 2;
    }
    int dims[4];
    for (int d = 0; d < 4; ++d) dims[d] = atoi(argv[2 + d]);
    const double omega = atof(argv[6]);
    const size_t V = (size_t)dims[0] * dims[1] * dims[2] * dims[3];
    const size_t n = V * 72;
    double *links = (double *)malloc(n * sizeof(double));
    if (!links) return 1;
    FILE *f = fopen(argv[7], "rb");
    if (!f || fread(links, sizeof(double), n, f) != n) {
        fprintf(stderr, "cannot read %zu doubles from %s\n", n, argv[7]);
        free(links);
        if (f) fclose(f);
        return 1;
    }
    fclose(f);
    lgf_lattice *h = NULL;
    double F = 0.0, theta = 0.0;
    int rc = 1;
    if (expect("create", lgf_create(dims, LGF_FP64_18, NULL, NULL, 0, &h), LGF_OK)) goto out;
    if (expect("load", lgf_load_links(h, links, n), LGF_OK)) goto out;
    if (expect("sweep", lgf_sweep(h, 2, omega, 0.0, 0, 0), LGF_OK)) goto out;
    if (expect("measure", lgf_measure(h, &F, &theta), LGF_OK)) goto out;
    if (expect("store", lgf_store_links(h, links, n), LGF_OK)) goto out;
    f = fopen(argv[8], "wb");
    if (!f || fwrite(links, sizeof(double), n, f) != n) {
        fprintf(stderr, "cannot write %s\n", argv[8]);
        if (f) fclose(f);
        goto out;
    }
    fclose(f);
    printf("%.17g %.17g\n", F, theta);
    rc = 0;
out:
    if (expect("destroy", lgf_destroy(h), LGF_OK)) rc = 1;
    free(links);
    return rc;
}

int main(int argc, char **argv)
{
    if (argc >= 2 && strcmp(argv[1], "check") == 0) return check();
    if (argc >= 2 && strcmp(argv[1], "run") == 0) return run(argc, argv);
    fprintf(stderr, "usage: abi_client check | run Lt Lz Ly Lx omega in.bin out.bin\n");
    return 2;
}
