"""Pins of the oracle's pair-list validity check (Sec. 2.3, Alg. alg_validity_check).

  * large-displacement check (LDC) against the strict expiry condition
    (eq. eq_strict_condition) by brute force over all pairs: LDC "valid" always
    implies strictly valid, and when every particle is a member the two agree;
  * the member count equals an independent count of particles whose
    displacement exceeds (rs - rc) - max displacement;
  * a hand-made two-particle case: an unlisted pair closing in below rc
    invalidates the list, one stopping short of rc does not, a listed pair never
    does;
  * DUTC: with force-free particles at speed u the first LDC check comes when
    the buffer rs - rc minus 2 u dt per step is no longer positive;
  * a whole run with DUTC + LDC gives the same trajectory as the half-skin rule
    (a missed pair would change the forces) with fewer rebuilds.
"""

import numpy as np
import pytest

import lj_inputs as li

RC, RS = 2.5, 2.8


def _min_image(d, L):
    return d - L * np.rint(d / L)


def _strict_valid(q, qold, L):
    """Brute force of the strict condition: no pair with old distance >= rs
    (not listed) and new distance < rc."""
    n = q.shape[0]
    for i in range(n):
        do = _min_image(qold[i + 1:] - qold[i], L)
        dn = _min_image(q[i + 1:] - q[i], L)
        if np.any((np.sum(do * do, axis=1) >= RS * RS) & (np.sum(dn * dn, axis=1) < RC * RC)):
            return False
    return True


def _perturbed(seed, n_fcc=4, amp=0.05, big=0.0, nbig=0):
    q0, L = li.jittered_fcc(n_fcc, amp=0.2, seed=seed)
    rng = np.random.default_rng(seed + 100)
    d = amp * rng.standard_normal(q0.shape)
    if nbig:
        idx = rng.choice(q0.shape[0], nbig, replace=False)
        d[idx] += big * rng.standard_normal((nbig, 3))
    return li.wrap_into_box(q0 + d, L), q0, L


def _case(seed):
    amp = [0.02, 0.04, 0.07, 0.1][seed % 4]
    big = [0.0, 0.15, 0.3][(seed // 4) % 3]
    return _perturbed(seed, amp=amp, big=big, nbig=(seed % 3) + 1 if big else 0)


def test_ldc_sound_and_exact_when_all_are_members(ref):
    kinds = set()
    for seed in range(24):
        q, qold, L = _case(seed)
        ok, nld, dm2 = ref.ldc_check(q, qold, L, RC, RS, ldc_max=10 ** 6)
        strict = _strict_valid(q, qold, L)
        if ok:
            assert strict, seed
        t = (RS - RC) - np.sqrt(dm2) - 1e-12
        if t < 0:
            assert nld == q.shape[0] and ok == strict, seed
        kinds.add((ok, t < 0, 0 < nld < q.shape[0]))
    # the cases cover: valid with some members, valid with all, invalid with all
    assert {(True, False, True), (True, True, False), (False, True, False)} <= kinds


@pytest.mark.parametrize("seed", range(6))
def test_ldc_member_count(ref, seed):
    q, qold, L = _perturbed(seed, amp=0.05)
    _, nld, dm2 = ref.ldc_check(q, qold, L, RC, RS, ldc_max=10 ** 6)
    d = _min_image(q - qold, L)
    disp = np.sqrt(np.sum(d * d, axis=1))
    assert dm2 == pytest.approx(disp.max() ** 2, rel=1e-12)
    thr = (RS - RC) - disp.max()
    assert nld == int(np.sum(disp > thr))
    # above the cap the list is invalid outright
    ok, nld2, _ = ref.ldc_check(q, qold, L, RC, RS, ldc_max=max(nld - 1, 0))
    if nld > 0:
        assert not ok and nld2 == nld


def test_ldc_two_particles(ref):
    L = np.array([12.0, 12.0, 12.0])
    qold = np.array([[3.0, 6.0, 6.0], [5.85, 6.0, 6.0], [3.0, 1.0, 1.0], [5.7, 1.0, 1.0]])
    # pair (0, 1) starts unlisted (2.85 >= rs), pair (2, 3) listed (2.7 < rs)
    close = qold.copy()
    close[0, 0] += 0.2
    close[1, 0] -= 0.2          # 2.45 < rc: a missed interaction
    ok, nld, _ = ref.ldc_check(close, qold, L, RC, RS)
    assert not ok and nld == 2
    short = qold.copy()
    short[0, 0] += 0.15
    short[1, 0] -= 0.15         # 2.55 > rc: still harmless
    assert ref.ldc_check(short, qold, L, RC, RS)[0]
    listed = qold.copy()
    listed[2, 0] += 0.2
    listed[3, 0] -= 0.2         # a listed pair may come as close as it likes
    assert ref.ldc_check(listed, qold, L, RC, RS)[0]


def test_dutc_first_check(ref):
    # two particles far apart: no force, constant speed u along x
    L = np.array([30.0, 30.0, 30.0])
    q = np.array([[5.0, 5.0, 5.0], [20.0, 20.0, 20.0]])
    u, dt, steps = 1.0, 0.005, 60
    v = np.array([[u, 0.0, 0.0], [0.0, -u, 0.0]])
    _, _, _, _, st = ref.run(q, v, L, steps, dt=dt, rc=RC, rs=RS, sample_every=0, rule="dutc_ldc",
                             full_stats=True)
    buf, first = RS - RC, None
    for k in range(1, steps + 1):
        buf -= 2.0 * np.sqrt(u * u) * dt
        if not buf > 0.0:
            first = k
            break
    assert st["ldc_checks"] == steps - first + 1
    assert st["rebuilds"] == 0 and st["ldc_kept"] == st["ldc_checks"]


@pytest.mark.parametrize("T", [1.0, 3.0])
def test_dutc_ldc_run_equals_half_skin_run(ref, T):
    q, L = li.fcc_lattice(6)
    v = li.maxwell_boltzmann(q.shape[0], T=T, seed=9)
    a = ref.run(q, v, L, 150, sample_every=10, full_stats=True)
    b = ref.run(q, v, L, 150, sample_every=10, rule="dutc_ldc", full_stats=True)
    assert np.abs(a[2] - b[2]).max() <= 1e-12 * np.abs(a[2]).max()
    assert np.abs(_min_image(a[0] - b[0], L)).max() < 1e-10
    assert b[4]["rebuilds"] < a[4]["rebuilds"]
    assert b[4]["ldc_checks"] > 0
