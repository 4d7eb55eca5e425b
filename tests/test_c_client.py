"""The C ABI from a plain C99 program (tests/c_client/folty_client.c).

* CPU: the header compiles as strict C99 with warnings as errors, the program
  links against libfolty.so, and without a GPU the first call fails loudly with
  FOLTY_EDEVICE (no CPU fallback).
* GPU: the program's counts, pairs, |Sol|, exists-exists-exists triples and
  vertex-query answers equal the hand-derived golden values.
"""
import json
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c_client", "folty_client.c")
LIBDIR = os.path.join(ROOT, "paper_2507_17215_amd")
GOLD = os.path.join(ROOT, "tests", "golden")


def build_client(tmp_path):
    exe = str(tmp_path / "folty_client")
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
           SRC, "-o", exe, "-L", LIBDIR, "-lfolty", f"-Wl,-rpath,{LIBDIR}", "-Wl,--allow-shlib-undefined"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def run_client(exe, n, edges, lines):
    text = f"{n} {len(edges)}\n" + "".join(f"{u} {v} {t}\n" for u, v, t in edges) + "".join(l + "\n" for l in lines)
    return subprocess.run([exe], input=text, capture_output=True, text=True, timeout=120)


def test_c_client_compiles_links_and_fails_loudly_without_gpu(tmp_path):
    from tests.conftest import gpu_available
    exe = build_client(tmp_path)
    if gpu_available():
        pytest.skip("a GPU is present")
    p = run_client(exe, 3, [(0, 1, 0), (0, 2, 1), (1, 2, 2)], ["Q 10 1 2 0 0 0"])
    assert p.returncode == 2
    assert p.stderr.startswith("ERROR -4 load")


@pytest.mark.gpu
def test_c_client_matches_golden_values(tmp_path):
    exe = build_client(tmp_path)
    d = json.load(open(os.path.join(GOLD, "hand_cases.json")))
    for g in d["graphs"]:
        lines = [f"Q {c['delta']} {c['theta'][0]} {c['theta'][1]} {c['variant']} {c.get('universe', 0)} "
                 f"{c.get('exclude_other', 0)}" for c in g["cases"]]
        p = run_client(exe, g["n"], g["edges"], lines)
        assert p.returncode == 0, p.stderr
        out = p.stdout.splitlines()
        pos = 0
        for c in g["cases"]:
            assert out[pos] == "COUNTS" + "".join(f" {x}" for x in c["counts"]), (g.get("name"), c)
            k = int(out[pos + 1].split()[1])
            pairs = [[int(x) for x in out[pos + 2 + i].split()] for i in range(k)]
            assert pairs == c["pairs"]
            assert out[pos + 2 + k] == f"NCERT {c['n_certificates']}"
            pos += 3 + k
    t = json.load(open(os.path.join(GOLD, "triad_cases.json")))
    lines = [f"T {c['delta']} {c['variant']} 7" for c in t["cases"]]
    p = run_client(exe, t["graph"]["n"], t["graph"]["edges"], lines)
    assert p.returncode == 0, p.stderr
    out = p.stdout.splitlines()
    pos = 0
    for c in t["cases"]:
        ns, ni = (int(x) for x in out[pos].split()[1:])
        assert ns == len(c["triples"]) and ni == sum(c["instances"])
        assert [[int(x) for x in out[pos + 1 + i].split()] for i in range(ns)] == c["triples"]
        assert out[pos + 1 + ns] == "INST" + "".join(f" {x}" for x in c["instances"])
        pos += 2 + ns
    v = json.load(open(os.path.join(GOLD, "vertex_cases.json")))
    lines = []
    for c in v["cases"]:
        inner = 1 if c["inner"] == "exists" else 0
        it = c.get("inner_theta", [1, 1])
        lines.append(f"V {c['delta']} {c['theta'][0]} {c['theta'][1]} {inner} {it[0]} {it[1]} 0")
    p = run_client(exe, v["graph"]["n"], v["graph"]["edges"], lines)
    assert p.returncode == 0, p.stderr
    out = p.stdout.splitlines()
    pos = 0
    for c in v["cases"]:
        k = int(out[pos].split()[1])
        got = [[int(x) for x in out[pos + 1 + i].split()] for i in range(k)]
        assert got == [[a, b] for a, b in zip(c["vertices"], c["good"])], c
        pos += 1 + k
