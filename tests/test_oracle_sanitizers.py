"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
every oracle entry point on random small graphs, all predicate codes and windows
(including one near 2^62), must run without a sanitizer report."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = textwrap.dedent("""
    import sys
    sys.path.insert(0, {root!r})
    import numpy as np
    import oracle.oracle as oo
    oo._LIB = {lib!r}
    oo.build = lambda force=False: oo._LIB
    from oracle.oracle import Oracle
    from paper_2507_17215_amd import synth
    rng = np.random.default_rng(5)
    for it in range(60):
        g = synth.random_small(rng, n_max=20, m_max=150, t_max=30)
        o = Oracle(g.n, g.src, g.dst, g.t, threads=2)
        for v in range(8):
            for d in (0, 3, 1 << 62):
                o.counts(d, v)
                o.triad_instances(d, v)
                o.triad_solutions(d, v)
                if g.m:
                    o.triad_pair(int(g.src[0]), int(g.dst[0]), d, v)
        o.counts_pool([0, 5, 10], 0)
        o.sizes()
        o.core_numbers()
        o.common_counts(np.arange(g.m))
    print("sanitizers clean")
""")


def test_oracle_under_sanitizers(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("libasan is not available")
    lib = str(tmp_path / "libfolty_oracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-shared", "-fPIC",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "folty_oracle.c"), "-o", lib],
                   check=True, capture_output=True, text=True)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    p = subprocess.run([sys.executable, "-c", DRIVER.format(root=ROOT, lib=lib)], env=env,
                       capture_output=True, text=True, timeout=600)
    assert p.returncode == 0, p.stderr[-3000:]
    assert "sanitizers clean" in p.stdout
    assert "runtime error" not in p.stderr
