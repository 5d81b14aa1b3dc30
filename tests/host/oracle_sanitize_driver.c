/* Host driver for the sanitizer run of the oracle (test infrastructure).
 *
 * Reads one scene and one workload from a binary file written by the test,
 * runs the oracle's entry points on it single-threaded (the whole method,
 * the per-ray trace, order-1 diffraction, wedges, every launch grid) and
 * prints the result counts.  Built with AddressSanitizer and
 * UndefinedBehaviorSanitizer, so any out-of-bounds access, leak or undefined
 * operation ends the run with a report and a non-zero status. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "sbr_oracle.h"

static void* rd(FILE* f, size_t bytes)
{
    void* p = malloc(bytes ? bytes : 1);
    if (!p || fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short read\n");
        exit(2);
    }
    return p;
}

int main(int argc, char** argv)
{
    if (argc != 2) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t* hdr = (int64_t*)rd(f, 8 * sizeof(int64_t));
    int64_t T = hdr[0], n_mat = hdr[1], n_rx = hdr[2];
    int32_t K = (int32_t)hdr[3], n = (int32_t)hdr[4], iters = (int32_t)hdr[5];
    int32_t sub = (int32_t)hdr[6];
    double* tri_v = (double*)rd(f, sizeof(double) * 9 * (size_t)T);
    int32_t* face = (int32_t*)rd(f, sizeof(int32_t) * (size_t)T);
    int32_t* mat = (int32_t*)rd(f, sizeof(int32_t) * (size_t)T);
    double* er = (double*)rd(f, sizeof(double) * (size_t)n_mat);
    double* ei = (double*)rd(f, sizeof(double) * (size_t)n_mat);
    double* tx = (double*)rd(f, sizeof(double) * 3);
    double* rx = (double*)rd(f, sizeof(double) * 3 * (size_t)n_rx);
    double* target = (double*)rd(f, sizeof(double));
    fclose(f);

    orc_params P = {K, n, iters, sub, *target, 28e9, 0.0, 1, 1, ORC_LAUNCH_EQUIANGULAR};
    orc_candidate *c = NULL, *u = NULL;
    orc_path* p = NULL;
    int64_t nc = 0, nu = 0, np = 0;
    int rc = orc_run(tri_v, face, mat, T, er, ei, (int32_t)n_mat, tx, rx, (int32_t)n_rx, &P, &c,
                     &nc, &u, &nu, &p, &np);
    if (rc) return 3;
    printf("events=%lld unique=%lld paths=%lld\n", (long long)nc, (long long)nu, (long long)np);

    /* steps 3-4 again from the winners, and path test 1 alone */
    orc_path* q = (orc_path*)malloc(sizeof(orc_path) * (size_t)(nu ? nu : 1));
    if (orc_path_records(tri_v, face, mat, T, er, ei, (int32_t)n_mat, tx, rx, (int32_t)n_rx, &P,
                         u, nu, q))
        return 3;
    orc_candidate* w = NULL;
    int64_t nw = 0;
    if (orc_path_test1(c, nc, &w, &nw) || nw != nu) return 3;
    orc_free(w);
    free(q);

    /* per-ray trace of every launch ray */
    int64_t R = orc_num_rays(n);
    int32_t* ot = (int32_t*)malloc(sizeof(int32_t) * (size_t)(R * (K + 1)));
    int32_t* of = (int32_t*)malloc(sizeof(int32_t) * (size_t)(R * (K + 1)));
    double* tt = (double*)malloc(sizeof(double) * (size_t)(R * (K + 1)));
    if (orc_trace_rays(tri_v, face, T, tx, n, ORC_LAUNCH_EQUIANGULAR, K, NULL, R, 1, ot, of, tt))
        return 3;
    free(ot); free(of); free(tt);

    /* every launch method */
    for (int32_t m = 0; m <= ORC_LAUNCH_EQUIDISTANT_OCTA; ++m) {
        int64_t Rm = orc_num_rays_m(m, n);
        double* d = (double*)malloc(sizeof(double) * 3 * (size_t)Rm);
        if (orc_launch_dirs_m(m, n, NULL, Rm, d)) return 3;
        free(d);
    }

    /* order-1 diffraction */
    int64_t nwg = orc_wedges(tri_v, face, T, NULL, 0);
    if (nwg < 0) return 3;
    double* wg = (double*)malloc(sizeof(double) * 17 * (size_t)(nwg ? nwg : 1));
    orc_wedges(tri_v, face, T, wg, nwg);
    free(wg);
    orc_candidate *dc = NULL, *du = NULL;
    orc_dpath* dp = NULL;
    int64_t ndc = 0, ndu = 0, ndp = 0;
    if (orc_diffract(tri_v, face, T, tx, rx, (int32_t)n_rx, &P, &dc, &ndc, &du, &ndu, &dp, &ndp))
        return 3;
    printf("wedges=%lld devents=%lld dpaths=%lld\n", (long long)nwg, (long long)ndc,
           (long long)ndp);

    orc_free(c); orc_free(u); orc_free(p);
    orc_free(dc); orc_free(du); orc_free(dp);
    free(hdr); free(tri_v); free(face); free(mat); free(er); free(ei); free(tx); free(rx);
    free(target);
    return 0;
}
