"""The host C code of the test infrastructure (the keyword-search and
peeling oracles, the input generators) built with AddressSanitizer and
UndefinedBehaviorSanitizer, then run against the brute-force pins, the
hand-derived goldens and the peeling re-simulation in a child process.
Any out-of-bounds access, use after free or undefined behaviour aborts the
child and fails the test. CPU only (gcc; no device code is built here).
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent(r"""
    import ctypes as C, json, os, sys
    sys.path.insert(0, ROOT); sys.path.insert(0, os.path.join(ROOT, "tests"))
    import numpy as np
    import oracle
    from synth import gen, tiny, workloads
    gen._LIB = SYN_LIB                       # the sanitized builds replace the plain ones
    oracle._lib = oracle._bind(C.CDLL(ORC_LIB))
    import brute
    from test_oracle_pins import _as_dict
    import test_peel_pins as pp

    # keyword search: brute force on random tiny graphs and the worked examples
    for seed in range(0, 400, 5):
        g = tiny.random_graph(seed)
        o = oracle.Oracle(g)
        D = brute.all_pairs(g)
        for q in tiny.random_queries(g, seed):
            want = brute.search(g, q.kw, q.d_max, q.k, D)
            want["edges"] = [[list(e) for e in es] for es in want["edges"]]
            assert _as_dict(o.search(q.kw, q.d_max, q.k)) == want, (seed, q)
        o.close()
    spec = json.load(open(os.path.join(ROOT, "tests", "golden", "worked_examples.json")))
    for case in spec["cases"]:
        g = tiny.from_edges(case["n"], case["edges"], case["labels"], case["n_labels"],
                            case["type_parent"], case["name"])
        o = oracle.Oracle(g)
        for q in case["queries"]:
            assert _as_dict(o.search(q["kw"], q["d_max"], q["k"])) == q["expect"]
    # the generators at a small scale, with the type tree, and a search on them
    g, qs = workloads.rmat24_hier(12, 32)
    o = oracle.Oracle(g)
    for q in qs:
        o.search(q.kw, q.d_max, q.k)
    g = workloads.chunglu10k()
    workloads.chunglu10k_queries(8)
    # peeling: the exact re-simulation, the FD golden, the optimised modes
    pp.test_fd_golden_hand_derived()
    pp.test_threshold_below_two_is_rejected()
    for seed in range(0, 40, 4):
        n, src, dst, ew, vw = pp.random_graph(seed, n_max=14, p_max=0.4)
        for metric in oracle.METRICS:
            c, a = oracle.metric_weights(metric, src, dst, n, ew, vw)
            oracle.peel(n, src, dst, c, a, 2, 1, 10)
            for mode in ("gpo", "lpo"):
                oracle.peel_opt(n, src, dst, c, a, 2, 1, 10, mode=mode)
            oracle.peel_sequential(n, src, dst, c, a)
    assert gen._L()._name == SYN_LIB and oracle.load()._name == ORC_LIB
    print("SANITIZED_OK", flush=True)
""")


def _gcc_lib(tmp, name, sources, extra):
    out = os.path.join(tmp, name)
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-shared", "-fPIC", "-o", out] + sources + extra + ["-lm"]
    subprocess.check_call(cmd)
    return out


def test_oracle_and_generators_under_asan_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc has no AddressSanitizer runtime here")
    tmp = str(tmp_path)
    orc = _gcc_lib(tmp, "liboracle_san.so",
                   [os.path.join(ROOT, "oracle", "kws_oracle.c"), os.path.join(ROOT, "oracle", "peel_oracle.c")], [])
    syn = _gcc_lib(tmp, "libsynth_san.so", [os.path.join(ROOT, "synth", "synth.c")], ["-fopenmp"])
    script = os.path.join(tmp, "child.py")
    with open(script, "w") as f:
        f.write(f"ROOT = {ROOT!r}\nORC_LIB = {orc!r}\nSYN_LIB = {syn!r}\n" + CHILD)
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "2"
    r = subprocess.run([sys.executable, script], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "SANITIZED_OK" in r.stdout, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
