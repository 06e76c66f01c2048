"""CPU tests of the C-ABI library: exported symbols, and the host-only entry
points (filter construction, KPM count, slicer) against the oracle."""
import json
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import paper_1802_05215_amd as ev

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")))


def _declared():
    txt = open(os.path.join(ROOT, "include", "evsl_mi355.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(evsl_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    ev.load()
    decl = _declared()
    assert sorted(ev.EXPORTS) == decl
    out = subprocess.run(["nm", "-D", "--defined-only", ev.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    have = set(re.findall(r"\bT (evsl_[a-z0-9_]+)", out))
    assert set(decl) <= have, set(decl) - have


INTERVALS = [
    ([1.0, 1.6, 0.0117, 7.9883], 1), ([1.0, 1.6, 0.0117, 7.9883], 2),
    ([0.6, 0.61, 0.4, 13.0], 1), ([0.6, 0.61, 0.4, 13.0], 2),
    ([-0.5, 0.2, -1.0, 3.0], 0), ([2.0, 2.9, 0.0, 3.0], 2),
    ([0.0, 0.5, 0.0, 12.0], 1), ([11.5, 12.0, 0.0, 12.0], 2),
    ([0.505, 0.509, 0.45, 13.0], 2), ([1.0, 1.005, 0.0, 7.9998], 1),
]


@pytest.mark.parametrize("intv,damp", INTERVALS)
def test_cheb_coeffs_match_oracle(intv, damp):
    p = ev.evsl_cheb_coeffs(intv, damping=damp, tau=0.8, tau_ext=0.4)
    q = oracle.find_pol(intv, damping=damp, tau=0.8, tau_ext=0.4)
    assert p.deg == q["deg"] and p.boundary == q["boundary"]
    assert abs(p.gamma - q["gamma"]) <= 1e-10
    assert abs(p.bar - q["bar"]) <= 1e-11
    # T_j(gamma) by recurrence vs cos(j acos gamma), and a one-ulp shift of gamma
    # (d T_j / d gamma = j U_{j-1}), both move coefficient j by O(j eps)
    assert np.abs(p.coef - q["coef"]).max() <= 5e-15 * (p.deg + 10) * np.abs(q["coef"]).max()
    assert p.cc == q["cc"] and p.dd == q["dd"]


def test_cheb_coeffs_reproduce_paper_degrees():
    for r in GOLD["lap_degrees"]["rows"] + GOLD["maxwell_degrees"]["rows"]:
        p = ev.evsl_cheb_coeffs([r["intv"][0], r["intv"][1], r["ab"][0], r["ab"][1]],
                                damping=ev.DAMP_SIGMA)
        assert abs(p.deg - r["deg"]) <= 1
    s = GOLD["slicing_49cube"]
    for row in s["rows"]:
        for (xi, eta), deg in zip(row["slices"], row["deg"]):
            assert ev.evsl_cheb_coeffs([xi, eta] + s["ab"], damping=ev.DAMP_SIGMA).deg == deg


def test_cheb_coeffs_errors():
    with pytest.raises(ev.EvslError) as e:
        ev.evsl_cheb_coeffs([1.0, 0.5, 0.0, 2.0])
    assert e.value.code == ev.EVSL_EINVAL
    with pytest.raises(ev.EvslError):
        ev.evsl_cheb_coeffs([0.0, 3.0, 0.0, 2.0])       # covers the whole spectrum
    p = ev.evsl_cheb_coeffs([1.0, 1.0001, 0.0, 8.0], max_deg=50)
    assert p.status == ev.EVSL_EDEGREE and p.deg == 50


def _moments(seed, K):
    rng = np.random.default_rng(seed)
    lam = np.sort(rng.uniform(0.2, 7.5, 3000))
    x = (lam - 4.0) / 4.0
    return np.array([np.cos(k * np.arccos(x)).sum() for k in range(K + 1)])


@pytest.mark.parametrize("damp", [0, 1, 2])
def test_kpm_count_and_slicer_match_oracle(damp):
    mom = _moments(3, 80)
    for (a, b) in [(0.5, 1.0), (0.0, 8.0), (3.3, 3.31), (-1.0, 2.0)]:
        c1 = ev.evsl_kpm_count(mom, damp, 0.0, 8.0, a, b)
        c2 = oracle.kpm_count(mom, damp, 0.0, 8.0, a, b)
        assert abs(c1 - c2) <= 1e-9 * max(1.0, abs(c2))
    for ns in (1, 2, 5, 10):
        s1 = ev.evsl_slice_spectrum(mom, damp, [0.5, 6.0, 0.0, 8.0], ns, 2000)
        s2 = oracle.slicer(mom, damp, [0.5, 6.0, 0.0, 8.0], ns, 2000)
        step = 5.5 / 1999
        assert np.all(np.abs(s1 - s2) <= step * 1.0001)
        assert s1[0] == 0.5 and s1[-1] == 6.0 and np.all(np.diff(s1) > 0)


def test_slicer_errors():
    mom = _moments(1, 20)
    with pytest.raises(ev.EvslError):
        ev.evsl_slice_spectrum(mom, 2, [1.0, 0.5, 0.0, 8.0], 3)
    with pytest.raises(ev.EvslError):
        ev.evsl_slice_spectrum(mom, 2, [0.0, 1.0, 0.0, 8.0], 10, npts=8)


@pytest.mark.parametrize("sigma", [0.0, 0.03])
def test_lanczos_count_and_slicer_match_oracle(sigma):
    """Host-only quadrature count and slicer of the library against the
    oracle's, on a quadrature the oracle computed (40x40 Laplacian)."""
    import evsl_inputs as I
    A = I.laplacian(40, 2)
    q = oracle.lanczos_dos(A, 40, 12, seed=4)
    for x0, x1 in ((1.0, 1.6), (0.0, 8.0), (2.5, 2.51), (-1.0, 0.5)):
        want = oracle.lanczos_count(q, A.n, sigma, x0, x1)
        got = ev.evsl_lanczos_count(q, A.n, sigma, x0, x1)
        assert abs(got - want) <= 1e-11 * A.n
    got = ev.evsl_slice_spectrum_lanczos(q, A.n, sigma, 1.0, 3.0, 6)
    want = oracle.lanczos_slicer(q, A.n, sigma, 1.0, 3.0, 6)
    assert np.array_equal(got, want)
    with pytest.raises(ev.EvslError):
        ev.evsl_lanczos_count(q, A.n, -1.0, 0.0, 1.0)


@pytest.mark.parametrize("kind", [0, 1])
def test_lspol_matches_oracle(kind):
    for lo, hi, deg in ((0.1, 1.0, 30), (1.0, 9.0, 12)):
        got = ev.evsl_lspol(kind, lo, hi, deg)
        want = oracle.lspol(kind, lo, hi, deg)
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    with pytest.raises(ev.EvslError):
        ev.evsl_lspol(kind, 0.0, 1.0, 5)


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every ctypes mirror of a header struct has the size and field offsets
    the C compiler gives the header's definition."""
    import ctypes as C

    import paper_1802_05215_amd as pk
    mirrors = {"evsl_csr_t": pk.CsrT, "evsl_pol_t": pk.PolT, "evsl_lan_opts_t": pk.LanOptsT,
               "evsl_si_opts_t": pk.SiOptsT, "evsl_eigs_t": pk.EigsT, "evsl_alloc_t": pk.AllocT}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "evsl_mi355.h"',
             'int main(void) {']
    for name, cls in mirrors.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            lines.append(f'  printf("{name} {f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n"):
        if ln:
            a, b, v = ln.split()
            got[(a, b)] = int(v)
    for name, cls in mirrors.items():
        assert got[(name, "size")] == C.sizeof(cls), name
        for f in cls._fields_:
            assert got[(name, f[0])] == getattr(cls, f[0]).offset, (name, f[0])
