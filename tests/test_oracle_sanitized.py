"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host
code only, gcc) runs edge cases cleanly and prints the ECCs the regular build
returns: size-1 axes, 2D to 4D, every dtype with NaN and infinities, 1 and
65535 bins, several threads, and the smoothing filter."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ecc_oracle.c")

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
int oracle_ecc(const void* data, int dtype, int ndim, const int64_t* dims, int32_t nbins,
               int construction, int range_mode, double lo, double hi, int threads, int64_t* ecc_out);
int oracle_smooth13(const float* in, float* out, int64_t n1, int64_t n2, const float* w);
/* argv: file dtype ndim d0 d1 d2 d3 nbins construction range_mode lo hi threads
 *   or: file smooth n1 n2 */
int main(int argc, char** argv)
{
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    fseek(f, 0, SEEK_END);
    long n = ftell(f);
    fseek(f, 0, SEEK_SET);
    char* buf = (char*)malloc(n > 0 ? (size_t)n : 1);
    if (fread(buf, 1, (size_t)n, f) != (size_t)n) return 3;
    fclose(f);
    if (argv[2][0] == 's') {
        int64_t n1 = atoll(argv[3]), n2 = atoll(argv[4]);
        float w[13];
        for (int k = 0; k < 13; ++k) w[k] = (float)(k + 1) / 91.0f;
        float* out = (float*)malloc((size_t)(n1 * n2) * sizeof(float));
        int rc = oracle_smooth13((const float*)buf, out, n1, n2, w);
        for (int64_t i = 0; i < n1 * n2; ++i) printf("%.9g\n", out[i]);
        free(out);
        free(buf);
        return rc;
    }
    int dtype = atoi(argv[2]), ndim = atoi(argv[3]);
    int64_t dims[4] = {atoll(argv[4]), atoll(argv[5]), atoll(argv[6]), atoll(argv[7])};
    int32_t nbins = atoi(argv[8]);
    int64_t* out = (int64_t*)malloc((size_t)nbins * sizeof(int64_t));
    int rc = oracle_ecc(buf, dtype, ndim, dims, nbins, atoi(argv[9]), atoi(argv[10]), atof(argv[11]),
                        atof(argv[12]), atoi(argv[13]), out);
    for (int32_t i = 0; i < nbins; ++i) printf("%lld\n", (long long)out[i]);
    free(out);
    free(buf);
    return rc;
}
"""


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    d = tmp_path_factory.mktemp("asan")
    drv = d / "driver.c"
    drv.write_text(DRIVER)
    exe = d / "oracle_asan"
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", "-pthread", str(drv), SRC, "-o", str(exe), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip(f"gcc cannot build with the sanitizers here: {r.stderr[-300:]}")
    return d, exe


def _run(sanitized, arr, args):
    d, exe = sanitized
    path = d / "case.bin"
    path.write_bytes(np.ascontiguousarray(arr).tobytes())
    # verify_asan_link_order=0: other libraries the environment preloads may come
    # before the ASan runtime
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe), str(path), *map(str, args)], capture_output=True, text=True, env=env,
                       timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-2000:]
    return r.stdout.split()


CASES = [
    # (shape, dtype, nbins, construction, range)
    ((1, 1), np.uint8, 256, "vertex", None),
    ((1, 7), np.uint8, 1, "top", None),
    ((5, 1, 4), np.uint16, 65535, "vertex", "auto"),
    ((6, 5, 4), np.uint16, 300, "top", (10, 40000)),
    ((3, 4, 2, 5), np.float32, 97, "vertex", "auto"),
    ((2, 3, 3, 2), np.float32, 50, "top", (-1.0, 1.0)),
    ((17, 23), np.float32, 4096, "vertex", (-2.0, 2.0)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_sanitized_oracle_matches(sanitized, case):
    import oracle
    shape, dtype, nbins, cons, rng = CASES[case]
    g = np.random.default_rng(700 + case)
    if dtype == np.float32:
        a = g.standard_normal(shape).astype(np.float32)
        flat = a.reshape(-1)
        if flat.size >= 4:
            flat[0], flat[1], flat[2] = np.nan, np.inf, -np.inf
    else:
        a = g.integers(0, 256 if dtype == np.uint8 else 65536, size=shape).astype(dtype)
    mode, lo, hi = (0, 0.0, 0.0) if rng is None else ((2, 0.0, 0.0) if rng == "auto" else (1,) + tuple(rng))
    dims = list(shape) + [1] * (4 - len(shape))
    for threads in (1, 3):
        got = _run(sanitized, a, [oracle.DTYPES[np.dtype(dtype)], len(shape), *dims, nbins,
                                  oracle.CONSTRUCTIONS[cons], mode, repr(float(lo)), repr(float(hi)), threads])
        want = oracle.ecc(a, nbins, cons, value_range=rng, threads=threads)
        assert [int(x) for x in got] == want.tolist(), (shape, dtype, threads)


def test_sanitized_smoothing(sanitized):
    import oracle
    a = np.random.default_rng(710).standard_normal((9, 14)).astype(np.float32)
    got = np.array([float(x) for x in _run(sanitized, a, ["s", 9, 14])], dtype=np.float32)
    w = (np.arange(1, 14, dtype=np.float32) / np.float32(91.0)).astype(np.float32)
    want = oracle.smooth13(a, w).reshape(-1)
    assert np.array_equal(got, want)
