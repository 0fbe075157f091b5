"""Pins for the oracle's self-boundness check (steps 9-10, Sec. 2.3).

- A shell of N particles in antipodal pairs at radius R: every particle sits at
  Phi = -G m N / R (the shell's own potential), so the escape speed is
  sqrt(2 G m N / R) in closed form.  Speeds on either side of it decide the
  outcome; removing the fast half lowers the escape speed of the rest by
  sqrt(1/2) (a cascade the iteration must follow); the 40% rule is exact
  (4 of 10 removed keeps the group, 6 of 10 discards it).
- A dense core and one outer particle: the outer particle is the outermost
  shell, Phi = -G m N / r, so it escapes exactly above sqrt(2 G m N / r).
- A pure-Python O(N^2) potential from the shell definition (every other
  member inside or at r_i counts as a point mass at the centre, every one
  outside as a shell at its own radius) and a round-by-round removal match the
  oracle on random groups.
- Galilean invariance (a common velocity changes nothing) and periodic
  unwrapping (a group across the box boundary behaves as in the interior).
- In the identification loop: only bound particles are claimed, a group that
  loses more than 40% claims nothing, and a compact clump of fast particles
  that passes steps 7-8 is discarded while the bound halos are claimed.
"""
import math

import numpy as np
import pytest

import synth
from oracle import cwthf as O

GM = 1.0e-3  # G m_p in (Mpc/h) (km/s)^2 for these hand-made groups


def _shell(k, R, centre, seed):
    rng = np.random.default_rng(seed)
    u = rng.normal(size=(k, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    dirs = np.concatenate([u, -u])  # antipodal pairs: the centre of mass is the centre
    return centre + R * dirs, dirs


def _shell_velocities(dirs, speeds, seed):
    # each pair moves with opposite velocities of the pair's speed, perpendicular-ish noise
    rng = np.random.default_rng(seed + 1)
    k = dirs.shape[0] // 2
    w = rng.normal(size=(k, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    v = w * np.asarray(speeds)[:, None]
    return np.concatenate([v, -v])


def test_shell_all_bound():
    L, k, R = 100.0, 20, 1.5
    x, dirs = _shell(k, R, np.array([40.0, 50.0, 60.0]), 1)
    vesc = math.sqrt(2 * GM * 2 * k / R)
    v = _shell_velocities(dirs, [0.5 * vesc] * k, 1)
    bound, kept, rounds = O.self_bound(x, v, L, np.arange(2 * k), np.array([40.0, 50.0, 60.0]), GM)
    assert bound.all() and kept and rounds == 1


@pytest.mark.parametrize("fast_pairs,kept_expect", [(2, True), (3, False)])
def test_forty_percent_rule_is_exact(fast_pairs, kept_expect):
    L, k, R = 100.0, 5, 2.0  # N0 = 10
    c0 = np.array([10.0, 20.0, 30.0])
    x, dirs = _shell(k, R, c0, 2)
    vesc = math.sqrt(2 * GM * 2 * k / R)
    speeds = [1.2 * vesc] * fast_pairs + [0.3 * vesc] * (k - fast_pairs)
    v = _shell_velocities(dirs, speeds, 2)
    bound, kept, rounds = O.self_bound(x, v, L, np.arange(2 * k), c0, GM)
    fast = np.array(speeds + speeds) > vesc
    assert (bound == ~fast).all()  # the slow ones stay bound at the lower escape speed
    assert kept == kept_expect and rounds == 2


def test_cascade_removes_everything():
    L, k, R = 100.0, 16, 1.0
    c0 = np.array([50.0, 50.0, 50.0])
    x, dirs = _shell(k, R, c0, 3)
    vesc = math.sqrt(2 * GM * 2 * k / R)
    v = _shell_velocities(dirs, [1.01 * vesc] * (k // 2) + [0.99 * vesc] * (k // 2), 3)
    bound, kept, rounds = O.self_bound(x, v, L, np.arange(2 * k), c0, GM)
    # round 1 removes the fast half; the rest now faces sqrt(1/2) of the escape speed
    assert not bound.any() and not kept and rounds == 2


@pytest.mark.parametrize("factor,bound_expect", [(0.98, True), (1.02, False)])
def test_outer_particle_escapes_above_its_closed_form_speed(factor, bound_expect):
    L = 100.0
    c0 = np.array([30.0, 30.0, 30.0])
    rng = np.random.default_rng(4)
    core = c0 + rng.normal(scale=1e-3, size=(400, 3))
    out = c0 + np.array([[0.8, 0.0, 0.0]])
    x = np.concatenate([core, out])
    n = x.shape[0]
    c = x.sum(axis=0) / n
    r = np.linalg.norm(out[0] - c)
    vesc = math.sqrt(2 * GM * n / r)  # the outermost shell: Phi = -G m N / r
    v = np.zeros_like(x)
    # its speed relative to the group's mean velocity is factor * vesc
    v[-1] = np.array([0.0, factor * vesc * n / (n - 1), 0.0])
    bound, kept, rounds = O.self_bound(x, v, L, np.arange(n), c0, GM)
    assert bound[:-1].all() and bool(bound[-1]) == bound_expect and kept


def _brute(x, v, ref, L, gm):
    d = [[(a - b + L / 2) % L - L / 2 if abs(a - b) >= L / 2 else a - b for a, b in zip(p, ref)] for p in x]
    alive = list(range(len(x)))
    rounds = 0
    while alive:
        rounds += 1
        m = len(alive)
        c = [sum(d[i][a] for i in alive) / m for a in range(3)]
        u = [sum(v[i][a] for i in alive) / m for a in range(3)]
        r = {i: math.sqrt(sum((d[i][a] - c[a]) ** 2 for a in range(3))) for i in alive}
        esc = []
        for i in alive:
            phi = 0.0
            for j in alive:  # inside or at (r_i, i): point mass at the centre; outside: its own shell
                phi -= gm / (r[i] if (r[j], j) <= (r[i], i) else r[j])
            s2 = sum((v[i][a] - u[a]) ** 2 for a in range(3))
            assert abs(s2 + 2 * phi) > 1e-9 * abs(2 * phi)  # the case is decided away from a tie
            if s2 > -2 * phi:
                esc.append(i)
        if not esc:
            break
        alive = [i for i in alive if i not in esc]
    return alive, rounds


@pytest.mark.parametrize("seed,n", [(5, 12), (6, 40), (7, 60), (8, 25)])
def test_matches_brute_force(seed, n):
    rng = np.random.default_rng(seed)
    L = 50.0
    ref = rng.random(3) * L
    x = (ref + rng.normal(scale=0.6, size=(n, 3))) % L  # may cross the boundary
    vesc_typ = math.sqrt(2 * GM * n / 0.6)
    v = rng.normal(scale=0.45 * vesc_typ, size=(n, 3))
    alive, rounds = _brute(x.tolist(), v.tolist(), ref.tolist(), L, GM)
    bound, kept, got_rounds = O.self_bound(x, v, L, np.arange(n), ref, GM)
    assert np.flatnonzero(bound).tolist() == alive and got_rounds == rounds
    assert kept == (5 * (n - len(alive)) <= 2 * n and len(alive) > 0)
    assert 0 < len(alive) < n  # the case removes some, keeps some


def test_galilean_invariance_and_periodic_unwrapping():
    rng = np.random.default_rng(9)
    L, n = 40.0, 50
    ref = np.array([1.0, 39.5, 20.0])  # near two faces
    x = (ref + rng.normal(scale=0.8, size=(n, 3))) % L
    v = rng.normal(scale=0.4 * math.sqrt(2 * GM * n / 0.8), size=(n, 3))
    a = O.self_bound(x, v, L, np.arange(n), ref, GM)
    b = O.self_bound(x, v + np.array([500.0, -300.0, 77.0]), L, np.arange(n), ref, GM)
    shift = np.array([18.0, -19.0, 0.5])  # the same group moved to the interior
    c = O.self_bound((x + shift) % L, v, L, np.arange(n), (ref + shift) % L, GM)
    for other in (b, c):
        assert (a[0] == other[0]).all() and a[1:] == other[1:]
    assert 0 < a[0].sum() < n


def _phase_box(seed=10):
    L, npt = 64.0, 120000
    pos, vel, m_p = synth.make_phase_box(L, npt, 25, "f32", seed)
    pos, vel = pos.numpy(), vel.numpy()
    # a compact clump of fast particles: dense enough for steps 7-8, not bound
    rng = np.random.default_rng(seed)
    clump = (np.array([32.0, 12.0, 50.0]) + rng.normal(scale=0.5, size=(4000, 3))).astype(np.float32) % L
    cv = rng.normal(scale=2.0e4, size=(4000, 3)).astype(np.float32)
    return np.concatenate([pos, clump]), np.concatenate([vel, cv]), L, m_p


def test_identification_loop_claims_bound_particles_only():
    pos, vel, L, m_p = _phase_box()
    n = 32
    kws = [n / (1000.0 * a) for a in (3.0, 2.0, 1.0)]
    gm = O.GRAV * m_p
    plain = O.identify(pos, L, n, kws, 4.0, 15)
    r = O.identify(pos, L, n, kws, 4.0, 15, vel=vel, grav_mass=gm)
    for i, (sp, sb) in enumerate(zip(plain["scales"], r["scales"])):
        assert (sb["bound_keep"] <= sb["keep"]).all()
        lab = sb["particle_label"]
        for k in np.flatnonzero(sb["keep"]):
            rt = int(sb["maxima"][k])
            claimed = np.flatnonzero(lab == rt)
            if not sb["bound_keep"][k]:
                assert claimed.size == 0
            else:
                assert claimed.size >= 15
                assert (r["halo_scale"][claimed] == i).all()
    # the clump (the last 4000 particles) is never claimed; bound halos are
    assert (r["halo_scale"][-4000:] == -1).all()
    assert (plain["halo_scale"][-4000:] >= 0).mean() > 0.5  # without the check the clump would be a halo
    assert 0 < (r["halo_scale"][:-4000] >= 0).sum() < (plain["halo_scale"][:-4000] >= 0).sum()


def test_removed_share_decides_the_group_in_the_loop():
    # every kept group of the loop claims exactly the members self_bound keeps,
    # and none when more than 40% of them leave
    pos, vel, L, m_p = _phase_box(11)
    n = 32
    kws = [n / (1000.0 * a) for a in (2.0, 1.0)]
    gm = O.GRAV * m_p
    r = O.identify(pos, L, n, kws, 4.0, 15, vel=vel, grav_mass=gm)
    free = np.ones(len(pos), dtype=bool)
    dropped = partial = 0
    for i, sc in enumerate(r["scales"]):
        cell = sc["cell_label"]
        raw = O.label(pos, L, n, cell)
        for k in np.flatnonzero(sc["keep"]):
            rt = int(sc["maxima"][k])
            members = np.flatnonzero((raw == rt) & free)
            ref = np.array([rt % n, (rt // n) % n, rt // (n * n)], dtype=float) * (L / n)
            bound, kept, _ = O.self_bound(pos, vel, L, members, ref, gm)
            ok = kept and bound.sum() >= 15
            assert bool(sc["bound_keep"][k]) == ok
            want = members[bound] if ok else np.zeros(0, dtype=np.int64)
            assert np.array_equal(np.flatnonzero(sc["particle_label"] == rt), want)
            dropped += int(not ok)
            partial += int(ok and not bound.all())
        free &= r["halo_scale"] != i
    assert dropped > 0 and partial > 0  # both outcomes occur: groups discarded, groups trimmed
