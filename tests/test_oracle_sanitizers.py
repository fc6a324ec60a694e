"""The oracle's C part under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only): a small C driver calls every exported routine on random
inputs, including the edge cases (n = 0, 1, a single i, every derivative
order, softening on and off, bad arguments), and must exit cleanly."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pairderiv.c")

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_pair_derivs(int64_t n, const double *mass, const double *path, int32_t K, double G, double eps2,
                       int64_t n_i, const int64_t *i_list, double *out, double *mag, double *nat);
int oracle_potential(int64_t n, const double *mass, const double *x, double G, double eps2, int64_t n_i,
                     const int64_t *i_list, double *phi);
int oracle_max_pair_rate(int64_t n, const double *mass, const double *x, double G, double eps2, double *qmax);

static double rnd(void) { return (double)rand() / RAND_MAX - 0.5; }

int main(void)
{
    srand(7);
    const int64_t sizes[] = {0, 1, 2, 17, 64};
    for (int si = 0; si < 5; ++si) {
        const int64_t n = sizes[si];
        for (int K = 0; K <= 5; ++K) {
            double *mass = malloc(sizeof(double) * (n + 1));
            double *path = malloc(sizeof(double) * (size_t)(K + 1) * 3 * (n + 1));
            double *out = malloc(sizeof(double) * (size_t)(K + 1) * 3 * (n + 1));
            double *mag = malloc(sizeof(double) * (size_t)(K + 1) * (n + 1));
            double *nat = malloc(sizeof(double) * (size_t)(K + 1) * (n + 1));
            double *phi = malloc(sizeof(double) * (n + 1));
            for (int64_t i = 0; i < n; ++i) mass[i] = 0.5 + rnd();
            for (int64_t e = 0; e < (K + 1) * 3 * n; ++e) path[e] = rnd();
            for (int s = 0; s < 2; ++s) {
                const double eps2 = s ? 1e-3 : 0.0;
                if (oracle_pair_derivs(n, mass, path, K, 1.0, eps2, 0, NULL, out, mag, nat) != 0) return 1;
                if (n > 0) {
                    const int64_t one = n - 1;
                    if (oracle_pair_derivs(n, mass, path, K, 1.0, eps2, 1, &one, out, mag, nat) != 0) return 2;
                }
                if (oracle_potential(n, mass, path, 1.0, eps2, 0, NULL, phi) != 0) return 3;
                double q = -1.0;
                if (oracle_max_pair_rate(n, mass, path, 1.0, eps2, &q) != 0) return 4;
            }
            free(mass); free(path); free(out); free(mag); free(nat); free(phi);
        }
    }
    /* bad arguments are refused, not dereferenced */
    double q;
    if (oracle_pair_derivs(-1, NULL, NULL, 1, 1.0, 0.0, 0, NULL, NULL, NULL, NULL) == 0) return 5;
    if (oracle_max_pair_rate(2, NULL, NULL, 1.0, 0.0, &q) == 0) return 6;
    printf("ok\n");
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", "-std=c99", str(drv), SRC, "-o", str(exe), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok"
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
