"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host code only),
driven through its entry points on a small graph: walks under every sampler and grouping,
the branching counter, hashed sources and the estimator (all edges, a query, push only, walks
only).  Any out-of-bounds access, leak or undefined behaviour fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "saba_oracle.c")

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int32_t orc_uniform_sources(const int32_t *, int32_t, int64_t, uint32_t, int32_t *);
int32_t orc_walks_histogram(const int32_t *, const int32_t *, int32_t, const int32_t *, int64_t,
                            int32_t, uint32_t, uint32_t, uint32_t, int32_t, int64_t *, int64_t *,
                            int32_t);
int32_t orc_distinct8(const int32_t *, const int32_t *, int32_t, const int32_t *, int64_t, int32_t,
                      uint32_t, uint32_t, uint32_t, int32_t, int32_t, int64_t *);
int32_t orc_walk_path(const int32_t *, const int32_t *, int32_t, int32_t, uint32_t, uint32_t,
                      int32_t *);
int32_t orc_aesc(const int32_t *, const int32_t *, int32_t, double, double, double, uint32_t,
                 uint32_t, uint32_t, int32_t, int32_t, int32_t, const int32_t *, int64_t, double *,
                 int32_t *, int32_t *, int64_t *, double *, double *, int64_t *, int64_t *,
                 double *, int32_t);

#define CHECK(x) do { if ((x) != 0) { fprintf(stderr, "failed: %s\n", #x); return 1; } } while (0)

int main(void) {
    /* circulant graph on 41 vertices with offsets 1 and 3 (4-regular, connected, odd cycles),
       plus vertex 41 with one edge to 0 and an isolated vertex 42 */
    enum { N = 43, C = 41 };
    int32_t *rp = calloc(N + 1, sizeof(int32_t)), *ci = malloc(sizeof(int32_t) * 4 * N);
    int32_t nnz = 0;
    for (int v = 0; v < N; ++v) {
        int32_t nb[6], k = 0;
        if (v < C) {
            int offs[4] = {C - 3, C - 1, 1, 3};
            for (int i = 0; i < 4; ++i) nb[k++] = (v + offs[i]) % C;
            if (v == 0) nb[k++] = 41;
        } else if (v == 41) {
            nb[k++] = 0;
        }
        for (int i = 0; i < k; ++i)  /* sort the row */
            for (int j = i + 1; j < k; ++j)
                if (nb[j] < nb[i]) { int32_t t = nb[i]; nb[i] = nb[j]; nb[j] = t; }
        for (int i = 0; i < k; ++i) ci[nnz++] = nb[i];
        rp[v + 1] = nnz;
    }
    const int64_t W = 3001;
    int32_t *src = malloc(sizeof(int32_t) * W);
    CHECK(orc_uniform_sources(rp, N, W, 7u, src));
    int64_t *ep = malloc(sizeof(int64_t) * N), *vi = malloc(sizeof(int64_t) * N), hist[9];
    for (int sm = 0; sm < 4; ++sm)
        for (int g = 0; g < 2; ++g) {
            CHECK(orc_walks_histogram(rp, ci, N, src, W, 9, 3u, g ? 8u : 1u, g ? 24u : 0u, sm, ep,
                                      vi, 2));
            CHECK(orc_distinct8(rp, ci, N, src, W, 9, 3u, g ? 8u : 1u, g ? 24u : 0u, sm, g, hist));
        }
    int32_t path[10];
    CHECK(orc_walk_path(rp, ci, 5, 9, 123u, 0u, path));
    /* the estimator on the connected part: vertices 0..41 (drop the isolated one) */
    const int32_t n2 = 42, m2 = rp[n2] / 2;
    double *sc = malloc(sizeof(double) * m2), *D = malloc(sizeof(double) * rp[n2]);
    double *MC = malloc(sizeof(double) * rp[n2]), *gv = malloc(sizeof(double) * rp[n2]);
    int32_t *tau = malloc(sizeof(int32_t) * rp[n2]), *ttau = malloc(sizeof(int32_t) * rp[n2]);
    int64_t *nreq = malloc(sizeof(int64_t) * rp[n2]), *v0 = malloc(sizeof(int64_t) * rp[n2]);
    int64_t *v1 = malloc(sizeof(int64_t) * rp[n2]);
    const int32_t query[6] = {0, 41, 3, 0, 7, 10};
    for (int mode = 0; mode < 4; ++mode) {
        const int32_t push_all = mode == 1, ttmax = mode == 2 ? 0 : -1;
        const int32_t *qq = mode == 3 ? query : NULL;
        CHECK(orc_aesc(rp, ci, n2, 0.5, 0.01, 0.6, 1u, mode == 3 ? 8u : 1u, mode == 3 ? 24u : 0u,
                       16, ttmax, push_all, qq, mode == 3 ? 3 : 0, sc, tau, ttau, nreq, D, MC, v0,
                       v1, gv, 2));
    }
    free(rp); free(ci); free(src); free(ep); free(vi); free(sc); free(D); free(MC); free(gv);
    free(tau); free(ttau); free(nreq); free(v0); free(v1);
    printf("ok\n");
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "driver"
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fopenmp",
                    "-ffp-contract=off", "-o", str(exe), SRC, str(drv), "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.strip() == "ok"
