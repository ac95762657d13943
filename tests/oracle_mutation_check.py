"""Mutation check of the oracle pins (run by hand on the CPU:
python tests/oracle_mutation_check.py).  Not collected by pytest.

Copies the tree the CPU suite needs (oracle/, tests/, workloads/, the
package with its built library, include/) into a temporary directory, checks
that the unmutated copy passes ``pytest -m "not gpu"``, then plants one
plausible mistake at a time in the copy's oracle and reruns that suite:
a mistake is CAUGHT when some pin fails.  The tracked sources are never
touched."""
import os
import shutil
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
muts = [
 ("oracle/orc_kernels.inc", "((REAL)701 / 294)", "((REAL)701 / 295)"),
 ("oracle/orc_kernels.inc", "return -1 + b * x * x - 5", "return -1 - b * x * x - 5"),
 ("oracle/orc_kernels.inc", "return -1 - b * x + (REAL)5 / 2 * (1 - t1);", "return -1 + b * x + (REAL)5 / 2 * (1 - t1);"),
 ("oracle/orc_kernels.inc", "series / 48 ", "series / 47 "),
 ("oracle/orc_kernels.inc", "(digit(delta, a + 1) ? -1 : 1)", "(digit(delta, a + 2) ? -1 : 1)"),
 ("oracle/orc_kernels.inc", "const REAL sign = (alpha % 2 == 1) ? 1 : -1;", "const REAL sign = 1;"),
 ("oracle/orc_kernels.inc", "(REAL)1 / 42};", "(REAL)1 / 41};"),
 ("oracle/orc_kernels.inc", "return 1 - 3 * t1;", "return 1 - 2 * t1;"),
 ("oracle/orc_algebra.inc", "const REAL ang = -2 * PI_R", "const REAL ang = 2 * PI_R"),
 ("oracle/orc_algebra.inc", "x[k + j + half] = w * (a - b) * h;", "x[k + j + half] = (a - b) * h;"),
 ("oracle/orc_algebra.inc", "for (int64_t half = 1; half < n; half *= 2)", "for (int64_t half = 1; half < n / 2; half *= 2)"),
 ("oracle/orc_algebra.inc", "x[k + j + half] = (a - b) * h;\n            }\n}", "x[k + j + half] = (b - a) * h;\n            }\n}"),
 ("oracle/orc_algebra.inc", "w[k] / (l + (REAL)sigma2)", "w[k] / (l - (REAL)sigma2)"),
 ("oracle/orc_algebra.inc", "const REAL sn = RSQRT((REAL)n);", "const REAL sn = (REAL)n;"),
 ("oracle/orc_algebra.c", "const double ang = -M_PI * (double)k / (double)n;\n                const double complex om = cos(ang) + sin(ang) * I;\n                const double complex a", "const double ang = M_PI * (double)k / (double)n;\n                const double complex om = cos(ang) + sin(ang) * I;\n                const double complex a"),
 ("oracle/orc_points.c", "if (digit) z += (t == 64) ? g[j] : (g[j] << (64 - t));", "if (digit) z += (t == 64) ? g[j] : (g[j] << (63 - t));"),
 ("oracle/orc_points.c", "acc += s_ts * col_bit(C[(size_t)j * m + k], s);", "acc += (int)((S[(size_t)j * 64 + s] >> (63 - t)) & 1u) * col_bit(C[(size_t)j * m + k], s);"),
 ("oracle/orc_points.c", "out[((size_t)r * cnt + ii) * d + j] = z ^ delta;", "out[((size_t)r * cnt + ii) * d + j] = z + delta;"),
 ("oracle/orc_points.c", "uint64_t orc_gray(uint64_t i) { return i ^ (i >> 1); }", "uint64_t orc_gray(uint64_t i) { return i ^ (i << 1); }"),
 ("oracle/orc_mll.c", "const double gk = 0.5 * p / (s * s) - 0.5 / s;", "const double gk = 0.5 * p / (s * s) + 0.5 / s;"),
 ("oracle/orc_mll.c", "L[r] = -0.5 * quad - 0.5 * logdet", "L[r] = -0.5 * quad + 0.5 * logdet"),
 ("oracle/orc_mll.c", "dlogs2[r] = sigma2 * gsum;", "dlogs2[r] = gsum;"),
 ("oracle/orc_mll.c", "rc = orc_transform(kind, lat ? -1 : 1, 1, m, in, out);", "rc = orc_transform(kind, 1, 1, m, in, out);"),
 ("oracle/orc_mll.c", "a[(size_t)r * n + j] = rn * (lat", "a[(size_t)r * n + j] = (lat"),
 ("oracle/orc_mll.c", "gr[j] += ai * zeta * t[j] * pre[j] * suf;", "gr[j] += ai * zeta * t[j] * suf;"),
 ("oracle/orc_mll.c", "gr[d] += ai * zeta * p;", "gr[d] += ai * p;"),
 ("oracle/orc_mll.c", "t[j] = gamma[j] * K;", "t[j] = K;"),
 ("oracle/__init__.py", "row = A[alpha * j + t % alpha, t // alpha, :]", "row = A[alpha * j + (t // alpha) % alpha, t % alpha, :]"),
 ("oracle/__init__.py", "row = A[alpha * j + t % alpha, t // alpha, :]", "row = A[j + t % alpha, t // alpha, :]"),
 ("oracle/__init__.py", "out[r, q] = I2 - 2.0 * np.dot(w, kappa)", "out[r, q] = I2 - np.dot(w, kappa)"),
 ("oracle/__init__.py", "return np.full(n, float(zeta)), float(zeta)", "return np.full(n, float(zeta)), 2.0 * float(zeta)"),
 ("oracle/__init__.py", "out[\"var\"][r] = I2 - np.dot(kappa, wk)", "out[\"var\"][r] = I2 + np.dot(kappa, wk)"),
 ("oracle/__init__.py", "out[\"s2\"][r] = np.dot(y[r], c) / n", "out[\"s2\"][r] = np.dot(y[r], c)"),
 ("oracle/__init__.py", "return zeta - 2.0 * zeta * omega.sum(axis=-1)", "return zeta - zeta * omega.sum(axis=-1)"),
 ("oracle/__init__.py", "s2=(y * c).sum(axis=-1) / n,", "s2=(y * c).sum(axis=-1),"),
 ("oracle/__init__.py", "return (1.0 + x @ np.asarray(c, np.float64)) ** (-(d + 1))", "return (1.0 + x @ np.asarray(c, np.float64)) ** (-d)"),
 ("oracle/__init__.py", "sigma = math.sqrt(((mu_r - mu) ** 2).sum() / (R - 1))", "sigma = math.sqrt(((mu_r - mu) ** 2).sum() / R)"),
 ("oracle/__init__.py", "t = float(stats.t.ppf(1.0 - tau / 2.0, R - 1))", "t = float(stats.t.ppf(1.0 - tau, R - 1))"),
 ("oracle/__init__.py", "return np.ldexp(np.asarray(words, dtype=np.uint64).astype(np.float64), -64)", "return np.ldexp(np.asarray(words, dtype=np.uint64).astype(np.float64), -63)"),
 ("oracle/__init__.py", "return np.cos(2.0 * np.pi * u + x @ np.asarray(c, np.float64))", "return np.cos(np.pi * u + x @ np.asarray(c, np.float64))"),
 ("oracle/orc_bpoints.c", "for (int k = 1; k < j; ++k) {", "for (int k = 0; k < j; ++k) {"),
 ("oracle/orc_bpoints.c", "for (int t = 0; t < T; ++t) v = v * (uint64_t)b + (uint64_t)z[t];", "for (int t = 0; t < T; ++t) v = v * (uint64_t)b + (uint64_t)z[T - 1 - t];"),
 ("oracle/orc_bpoints.c", "s += (long)S[t * BT_MAX + k] * z[k];", "s += (long)S[k * BT_MAX + t] * z[k];"),
 ("oracle/orc_bpoints.c", "z[t] = (z[t] + dl[t]) % b;", "z[t] = (z[t] + b - dl[t]) % b;"),
 ("oracle/orc_bpoints.c", "const uint64_t prefix = t == 1 ? 0 : z >> (65 - t);", "const uint64_t prefix = t == 1 ? 0 : z >> (64 - t);"),
 ("oracle/orc_bpoints.c", "const int b = kind == ORC_HALTON ? orc_nth_prime(j + 1) : base;", "const int b = kind == ORC_HALTON ? orc_nth_prime(j + 2) : base;"),
 ("oracle/orc_bpoints.c", "P[r * T + c] = (r == 0 || r == c) ? 1 % b : (P[(r - 1) * T + (c - 1)] + P[r * T + (c - 1)]) % b;", "P[r * T + c] = (r == 0 || r == c) ? 1 % b : (P[(r - 1) * T + (c - 1)] + 2 * P[r * T + (c - 1)]) % b;"),
]

res = []


def run_suite(cwd):
    r = subprocess.run([sys.executable, "-m", "pytest", "tests/", "-q", "-x", "-m", "not gpu",
                        "-p", "no:cacheprovider"], cwd=cwd, capture_output=True, text=True,
                       timeout=900)
    return r


def main():
    with tempfile.TemporaryDirectory(prefix="orc_mut_") as tmp:
        ign = shutil.ignore_patterns("__pycache__", "*.pyc", "liborc.so*", "_build", "*.o")
        for d in ("oracle", "tests", "workloads", "paper_2502_14256_amd", "include"):
            shutil.copytree(os.path.join(ROOT, d), os.path.join(tmp, d), ignore=ign)
        for f in ("pytest.ini",):
            shutil.copy(os.path.join(ROOT, f), tmp)
        base = run_suite(tmp)
        if base.returncode != 0:
            print(base.stdout[-3000:], base.stderr[-3000:])
            sys.exit("the unmutated copy does not pass the CPU suite: no mutation result is valid")
        print("baseline (unmutated copy):", base.stdout.strip().splitlines()[-1], flush=True)
        for f, a, b in muts:
            path = os.path.join(tmp, f)
            src = open(path).read()
            assert src.count(a) >= 1, (f, a)
            open(path, "w").write(src.replace(a, b, 1))
            try:
                r = run_suite(tmp)
                caught = r.returncode != 0
            finally:
                open(path, "w").write(src)
            res.append((caught, f, b[:60]))
            print("CAUGHT " if caught else "MISSED ", f, repr(b[:70]), flush=True)
    print(sum(c for c, _, _ in res), "of", len(res), "caught")


if __name__ == "__main__":
    main()
