"""Planted mistakes: each mutant of the oracle must fail at least one pin.

A copy of the oracle source gets one plausible mistake (a wrong index, a
flipped test, a dropped comparison, a wrong bit), is compiled into a temp
directory, and a subprocess runs a quick selection of the pins against it.
The mutant is "caught" when a pin fails or the process dies.  This shows the
pins of test_oracle_pins.py are sharp enough to notice such slips.
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "qms_oracle.c")

MUTANTS = {
    "merge_first_run_off_by_one": (
        "    swap_merge(a, src + h, h, dst, k);",
        "    swap_merge(a, src + h, k, dst, k);"),
    "larger_side_mergesorted": (
        "if (n_left < n / 2) {",
        "if (n_left >= n / 2) {"),
    "median_of_3_missing_third_exchange": (
        "    cmp_exchange(a, lo, m); /* key[lo] <= key[m] <= key[l] */",
        "    /* dropped */"),
    "merge_takes_wrong_head": (
        "            swap_ij(a, o, y);\n            y++;",
        "            swap_ij(a, o, y);\n            x++;"),
    "merge_window_run_misplaced": (
        "size_t x = x0, y = w + nx, o = w;",
        "size_t x = x0, y = w + ny, o = w;"),
    "total_order_positive_bit": (
        "return (u & KEY_SIGN) ? ~u : (u | KEY_SIGN);",
        "return (u & KEY_SIGN) ? ~u : u;"),
    "mom_upper_median": (
        "qkey_t p = med[(c - 1) / 2];",
        "qkey_t p = med[c / 2];"),
    "mom_triples_overlap": (
        "qkey_t x = keys[3 * i], y = keys[3 * i + 1], z = keys[3 * i + 2];",
        "qkey_t x = keys[2 * i], y = keys[2 * i + 1], z = keys[2 * i + 2];"),
    "mom_median_of_three_wrong": (
        "med[i] = z < lo ? lo : (z > hi ? hi : z);",
        "med[i] = z < lo ? z : (z > hi ? hi : z);"),
    "x_never_called": (
        "    if (n < a->xt) {",
        "    if (n < 2) {"),
    "x_recursion_includes_pivot": (
        "            clever_quicksort(a, lo, b);\n            lo = b + 1;",
        "            clever_quicksort(a, lo, b + 1);\n            lo = b + 1;"),
    "x_joint_movement_short": (
        "        swap_blocks(a, src, dst, n);",
        "        swap_blocks(a, src, dst, n - 1);"),
    "partition_scan_skips_element": (
        "        swap_ij(a, i, j);\n        i++;\n        j--;",
        "        swap_ij(a, i, j);\n        i += 2;\n        j--;"),
}

CHECK = textwrap.dedent(r"""
    import itertools, math, sys
    import numpy as np
    sys.path.insert(0, ROOT)
    import oracle
    oracle._LIB_PATH = LIB
    from tests.test_oracle_pins import qms_recurrence
    from paper_1804_10062_amd import inputs
    failures = []
    T = qms_recurrence(8)
    for n in range(2, 9):
        tot = cnt = 0
        for p in itertools.permutations(range(n)):
            s, _, c = oracle.sort(np.array(p, dtype=np.uint32))
            if s.tolist() != list(range(n)):
                failures.append(("perm", n)); break
            tot += c.comparisons; cnt += 1
        if abs(tot / cnt - T[n]) > 1e-9:
            failures.append(("avg", n))
    rng = np.random.default_rng(1)
    for n in (20, 37, 100, 1000):
        x = rng.permutation(n).astype(np.uint32)
        if oracle.sort(x)[0].tolist() != list(range(n)):
            failures.append(("rand", n))
    for seed in range(6):
        r = np.random.default_rng(seed)
        x = r.integers(0, 2**32, 101, dtype=np.uint64).astype(np.uint32)
        k, _, b, c = oracle.partition(x, 0, 101)
        med = sorted([int(x[0]), int(x[50]), int(x[100])])[1]
        if k[b] != med or c.comparisons != 101 or not (k[:b] <= k[b]).all():
            failures.append(("partition", seed))
    f = np.array([1.0, -1.0, 0.0, -0.0, 2.5, -3.0], dtype=np.float32)
    s = oracle.sort(f)[0]
    want = np.array([-3.0, -1.0, -0.0, 0.0, 1.0, 2.5], dtype=np.float32)
    if s.view(np.uint32).tolist() != want.view(np.uint32).tolist():
        failures.append(("f32",))
    from tests.test_oracle_pins import _mom_pivot_by_counting
    r = np.random.default_rng(7)
    for n in (4, 9, 10, 31):
        for _ in range(40):
            x = r.integers(0, 20, n).astype(np.uint32)
            if oracle.mom_pivot(x) != _mom_pivot_by_counting(x):
                failures.append(("mom", n)); break
    from tests.test_oracle_xsort import cqs_recurrence, msort_x_avg
    Q = cqs_recurrence(16)
    for n in range(2, 8):
        tot = cnt = 0
        for p in itertools.permutations(range(n)):
            s, _, c = oracle.clever_quicksort(np.array(p, dtype=np.uint32))
            if s.tolist() != list(range(n)):
                failures.append(("cqs perm", n)); break
            tot += c.comparisons; cnt += 1
        if abs(tot / cnt - Q[n]) > 1e-9:
            failures.append(("cqs avg", n))
    for xt in (5, 8):
        tot = cnt = 0
        buf = np.arange(50, 57, dtype=np.uint32)
        for p in itertools.permutations(range(7)):
            k, _, c = oracle.msort_x(np.concatenate([np.array(p, dtype=np.uint32), buf]), 0, 7, 7, xt)
            if k[7:].tolist() != list(range(7)):
                failures.append(("msort_x perm", xt)); break
            tot += c.comparisons; cnt += 1
        if abs(tot / cnt - msort_x_avg(7, xt, Q, {})) > 1e-9:
            failures.append(("msort_x avg", xt))
    for xt in (3, 17, None):
        x = rng.permutation(3000).astype(np.uint32)
        if oracle.sort_x(x, x_thresh=xt)[0].tolist() != list(range(3000)):
            failures.append(("sort_x", xt))
    print("FAILURES", failures)
    sys.exit(1 if failures else 0)
""")


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found"
    mutant_c = tmp_path / "mutant.c"
    mutant_c.write_text(src.replace(old, new))
    objs = []
    for bits in (32, 64):
        for counting in (1, 0):
            o = tmp_path / f"m{bits}_{counting}.o"
            subprocess.check_call(["gcc", "-std=c11", "-O1", "-fPIC", "-w",
                                   f"-DQMSO_COUNTING={counting}", f"-DQMSO_KEY_BITS={bits}",
                                   "-c", str(mutant_c), "-o", str(o)])
            objs.append(str(o))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-shared", "-o", str(lib)] + objs)
    script = f"ROOT = {ROOT!r}\nLIB = {str(lib)!r}\n" + CHECK
    r = subprocess.run([sys.executable, "-c", script], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0, f"mutant {name} passed every pin:\n{r.stdout}"


def test_unmutated_oracle_passes_the_same_checks(tmp_path):
    import oracle
    lib = oracle.build(force=False)
    script = f"ROOT = {ROOT!r}\nLIB = {lib!r}\n" + CHECK
    r = subprocess.run([sys.executable, "-c", script], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
