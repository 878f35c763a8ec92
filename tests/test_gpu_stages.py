"""Stage-chained parity at a flat 1e-12 per field: every RK4 stage the GPU
runs is checked against the oracle's single-stage function applied to the
GPU's OWN stage input (with the ghosts the GPU filled), its own u_n and its
own accumulator.  Each comparison is therefore one substep deep, so rounding
differences of earlier stages (the oracle sums the RK4 combination in
another order, and the stencils amplify ulp-level differences of O(1) fields
into noise-level fields over many substeps) cannot accumulate: the bar is the
flat 1e-12 of the float64 path, for the stage output and the accumulator.

Stage s (paper Sec. 2.2, classical RK4; E restores det gt = 1, tr At = 0):
    1: u1 = E(u + dt/2 k(u)),     acc = u + dt/6 k
    2: u2 = E(u + dt/2 k(u1)),    acc += dt/3 k
    3: u3 = E(u + dt k(u2)),      acc += dt/3 k
    4: u' = E(acc + dt/6 k(u3))
The cases cover the single-box path stage by stage, the persistent launch
over boxes whose bricks outnumber the resident blocks (every block walks
several bricks and reuses its LDS buffers), the batched plan replayed as a
HIP graph, and hierarchy patches whose stage inputs carry prolonged ghosts.
"""
import ctypes

import numpy as np
import pytest
import torch

from gpu_helpers import normrel, to_dev, to_host
from paper_2607_08743_amd import inputs as I
from paper_2607_08743_amd import z4c

pytestmark = pytest.mark.gpu
TOL = 1e-12
PERSISTENT = z4c.Tile(8, 8, 8, 2, 1)  # the benchmark's tile: one 512-thread block per CU, looping


def _ozp(oz, p):
    return oz.params(p.kappa1, p.kappa2, p.kappa3, p.eta, p.shift_coeff, p.ko_sigma, p.w_floor, p.lapse_uses_K)


def evolved_points(g, sample=None, seed=0):
    """(i, j, k) of the points a substep writes: the active points, every
    ghost of a Sommerfeld box, the ghosts at and above the plane of an
    equatorial box.  sample: that many random points (plus the 8 corners of
    the evolved region) instead of all of them."""
    N = g.shape[1:]  # (Nz, Ny, Nx)
    m = np.zeros(N, dtype=bool)
    if g.bc == I.BC_SOMMERFELD:
        m[:] = True
    elif g.bc == I.BC_EQUATORIAL:
        m[g.ng:] = True
    else:
        m = g.active_mask()
    kk, jj, ii = np.nonzero(m)
    pts = np.stack([ii, jj, kk], axis=1).astype(np.int32)
    if sample is not None and sample < len(pts):
        rng = np.random.default_rng(seed)
        lo, hi = pts.min(axis=0), pts.max(axis=0)
        corners = np.array([[a, b, c] for a in (lo[0], hi[0]) for b in (lo[1], hi[1]) for c in (lo[2], hi[2])],
                           dtype=np.int32)
        pts = np.concatenate([pts[rng.choice(len(pts), sample, replace=False)], corners])
    return pts


def _at(u, pts):
    return u[:, pts[:, 2], pts[:, 1], pts[:, 0]]


def check_stage(oz, ozp, g, stage, dt, src, un, acc_prev, out, acc, pts, label):
    """Stage output and accumulator of one substep against the oracle on the
    GPU's own inputs (host arrays), at the points pts.  The bar is 1e-12 per
    field, norm-relative; a field above it is held instead to the oracle's
    own one-ulp sensitivity for the same evaluation (its inputs perturbed by
    one ulp), where that is larger: a field whose stage values are a
    cancellation (Theta on puncture data, which starts at 0 and moves by dt
    times alpha/2 times the Hamiltonian constraint of data that solve it)."""
    gd = g.as_dict()
    c = {1: 0.5 * dt, 2: 0.5 * dt, 3: dt, 4: dt / 6.0}[stage]
    base = {1: src, 2: un, 3: un, 4: acc_prev}[stage]
    ref = oz.stage_points(src, base, c, gd, pts, ozp).T
    e = normrel(_at(out, pts), ref)
    has_acc = stage < 4 and acc is not None
    if has_acc:
        k = oz.rhs_points(src, gd, pts, ozp).T
        accb = src if stage == 1 else acc_prev
        ref_acc = _at(accb, pts) + (dt / 6.0 if stage == 1 else dt / 3.0) * k
        ea = normrel(_at(acc, pts), ref_acc)
    bound = bound_acc = np.full(e.shape, TOL)
    if e.max() > TOL or (has_acc and ea.max() > TOL):
        rng = np.random.default_rng(0)

        def pert(x):
            return x + np.spacing(x) * rng.choice([-1.0, 1.0], size=x.shape)
        src_p = pert(src)
        base_p = src_p if base is src else pert(base)
        bound = np.maximum(TOL, normrel(oz.stage_points(src_p, base_p, c, gd, pts, ozp).T, ref))
        if has_acc:
            accb_p = src_p if stage == 1 else pert(acc_prev)
            k_p = oz.rhs_points(src_p, gd, pts, ozp).T
            ref_acc_p = _at(accb_p, pts) + (dt / 6.0 if stage == 1 else dt / 3.0) * k_p
            bound_acc = np.maximum(TOL, normrel(ref_acc_p, ref_acc))
        del src_p, base_p
        over = np.nonzero((e > TOL) | ((ea > TOL) if has_acc else False))[0]
        print(f"{label} stage {stage}: fields above 1e-12 {list(over)}: normrel {e[over]}, "
              f"oracle one-ulp sensitivity {bound[over]}", flush=True)
    print(f"{label} stage {stage}: max per-field normrel output {e.max():.2e}"
          + (f", acc {ea.max():.2e}" if has_acc else ""), flush=True)
    if has_acc:
        assert np.all(ea <= bound_acc), (label, stage, "acc", ea, bound_acc)
    assert np.all(e <= bound), (label, stage, "u_out", e, bound)
    # the stage moved the state by much more than the tolerance (non-trivial comparison)
    moved = normrel(ref, _at(base, pts))
    assert moved.max() > 1e3 * TOL, (label, stage, moved)
    return max(e.max(), ea.max()) if has_acc else e.max()


def stage_chain(oz, g, u0, dt, nsteps, params=None, shell=None, pts=None, label=""):
    """Advance one box with apply_ghosts + rk4_substep (the rotation
    u -> A -> B -> A -> u of the single-box path) and check every stage."""
    params = params or z4c.default_params()
    ozp = _ozp(oz, params)
    u = to_dev(u0)
    a, b, acc = torch.empty_like(u), torch.empty_like(u), torch.zeros_like(u)
    sh = None if shell is None else to_dev(shell)
    pts = evolved_points(g) if pts is None else pts
    seq = ((u, a), (a, b), (b, a), (a, u))
    worst = 0.0
    for step in range(nsteps):
        for s, (src, dst) in enumerate(seq, start=1):
            z4c.apply_ghosts(src, g, sh)
            src_h, un_h, acc_h = to_host(src), to_host(u), to_host(acc)
            z4c.rk4_substep(s, dt, src, u, acc, dst, g, params)
            worst = max(worst, check_stage(oz, ozp, g, s, dt, src_h, un_h, acc_h, to_host(dst), to_host(acc),
                                           pts, f"{label} step {step}"))
    return worst, to_host(u)


def test_stages_plane_wave_noise(oz):
    print("case: stage chain, 32^3 periodic plane wave + noise, 2 steps", flush=True)
    g, u, dt = I.config_plane_wave()
    stage_chain(oz, g, u, dt, 2, label="plane wave")


def test_stages_strong_field_all_terms(oz):
    print("case: stage chain, 24^3 strong random field, kappa1/2/3 and lapse_uses_K set", flush=True)
    g = I.centered_grid(24, 0.1, bc=I.BC_PERIODIC)
    u = I.random_strong_field_state(g, seed=5)
    p = z4c.default_params(kappa1=0.3, kappa2=0.2, kappa3=0.7, lapse_uses_K=1)
    stage_chain(oz, g, u, 0.25 * g.h[0], 1, params=p, label="strong field")


def test_stages_punctures_sommerfeld(oz):
    print("case: stage chain, 24^3 punctures, Sommerfeld ghosts evolved, 2 steps", flush=True)
    g, u, dt = I.config_punctures(24)
    stage_chain(oz, g, u, dt, 2, label="punctures")


def test_stages_copy_box(oz):
    print("case: stage chain, 20x16x12 copy box with a noisy shell", flush=True)
    g = I.centered_grid((20, 16, 12), 0.25, center=(5.0, 0.0, 0.0), bc=I.BC_COPY)
    u = I.brill_lindquist_state(g)
    shell = I.shell_of(u, g) + np.random.default_rng(4).uniform(-1e-6, 1e-6, I.shell_of(u, g).shape)
    stage_chain(oz, g, u, 0.5 * g.h[0], 1, shell=shell, label="copy box")


def test_stages_equatorial(oz):
    print("case: stage chain, 24x24x12 equatorial half box", flush=True)
    g, u, dt = I.config_punctures_equatorial(24)
    stage_chain(oz, g, u, dt, 1, label="equatorial")


def test_stages_persistent_multibrick(oz):
    """72^3 punctures: 729 bricks of 8^3 against at most 256 resident
    blocks of the benchmark tile, so every block walks several bricks
    (persistent loop, LDS buffers reused between bricks).  Every stage is
    checked against the oracle on all evolved points; the step is then
    bitwise equal to the non-persistent launch."""
    print("case: stage chain, 72^3 punctures, persistent tile 8x8x8x2", flush=True)
    g, u, dt = I.config_punctures(72)
    try:
        z4c.select_tile(z4c.FP64, PERSISTENT)
        _, got_p = stage_chain(oz, g, u, dt, 1, label="persistent 72^3")
        st = z4c.Stepper(g, u, dt)
        st.step(1)
        got_p2 = to_host(st.u)
        del st
        z4c.select_tile(z4c.FP64, z4c.Tile(8, 8, 8, 2, 0))
        st = z4c.Stepper(g, u, dt)
        st.step(1)
        got_np = to_host(st.u)
        del st
    finally:
        z4c.select_tile(z4c.FP64, None)
    assert np.array_equal(got_p, got_p2)
    assert np.array_equal(got_p, got_np)
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", [z4c.FP64, z4c.MIXED])
def test_persistent_dma_register_bitwise(prec):
    """One stage of a 72^3 box, persistent and not, through the LDS-DMA
    staging and, with the field stride padded to an odd value, through the
    register staging: the persistent loop gives the bits of the
    non-persistent launch on both paths, and in float64 the two paths agree."""
    print(f"case: persistent DMA vs register staging vs non-persistent, 72^3, precision {prec}", flush=True)
    g, u, dt = I.config_punctures(72)
    L = z4c.lib()
    p = z4c.default_params(precision=prec)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    geo = (int(g.n[0]), int(g.n[1]), int(g.n[2]), int(g.ng))
    outs = []
    try:
        for pers, pad in ((1, 0), (1, 1), (0, 0), (0, 1)):
            z4c.select_tile(prec, z4c.Tile(8, 8, 8, 2, pers))
            sf = g.stored + pad
            du = torch.zeros((25, sf), dtype=torch.float64, device="cuda")
            du[:, :g.stored] = to_dev(u).reshape(25, -1)
            acc = torch.zeros_like(du)
            out = torch.full_like(du, float("nan"))
            z4c.check(L.rk4_substep(2, ctypes.c_double(dt), ctypes.c_void_p(du.data_ptr()),
                                    ctypes.c_void_p(du.data_ptr()), ctypes.c_void_p(acc.data_ptr()),
                                    ctypes.c_void_p(out.data_ptr()), ctypes.c_long(sf), *geo,
                                    ctypes.c_double(g.h[0]), ctypes.c_double(g.h[1]), ctypes.c_double(g.h[2]),
                                    ctypes.c_double(g.x0[0]), ctypes.c_double(g.x0[1]), ctypes.c_double(g.x0[2]),
                                    int(g.bc), ctypes.byref(p), stream), "rk4_substep")
            outs.append(to_host(out)[:, :g.stored])
            del du, acc, out
    finally:
        z4c.select_tile(prec, None)
    # persistent == non-persistent for each staging path
    assert np.array_equal(outs[0], outs[2])
    assert np.array_equal(outs[1], outs[3])
    if prec == z4c.FP64:
        # float64 tiles either way: the two staging paths agree bitwise (the
        # mixed register path rounds values, the DMA path differences)
        assert np.array_equal(outs[0], outs[1])
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n", [128, 256, 320])
def test_plan_persistent_stages(oz, n):
    """The benchmark's launch: a persistent plan (tile 8x8x8x2; 4096, 32768
    and 64000 bricks per launch against 256 resident blocks) over the n^3
    puncture box (256^3 is the benchmark's own box; at 320^3 each state array
    passes 2^32 bytes), one RK4 step replayed
    from the captured graph.  Stages 3 and 4 are read back from the plan's
    own buffers (B holds u2, A holds u3, the accumulator acc3) and checked
    against the oracle at sampled points; the whole step is bitwise equal to
    the non-persistent single-box path."""
    print(f"case: persistent plan {n}^3 punctures vs oracle stages 3, 4 and vs single-box path", flush=True)
    g, u, dt = I.config_punctures(n)
    ozp = _ozp(oz, z4c.default_params())
    plan = z4c.Plan([I.Box(g, u, None, dt)], tile=PERSISTENT)
    plan.step(1, use_graph=True)
    a, b, acc, _ = plan._keep[0]
    new, a_h, b_h, acc_h = to_host(plan.u[0]), to_host(a), to_host(b), to_host(acc)
    plan.close()
    del plan, a, b, acc
    torch.cuda.empty_cache()
    pts = evolved_points(g, sample=3000, seed=n)
    check_stage(oz, ozp, g, 3, dt, b_h, u, None, a_h, None, pts, f"plan {n}^3")
    check_stage(oz, ozp, g, 4, dt, a_h, None, acc_h, new, None, pts, f"plan {n}^3")
    del a_h, b_h, acc_h
    st = z4c.Stepper(g, u, dt)  # default tile: not persistent
    st.step(1)
    assert np.array_equal(to_host(st.u), new)
    del st
    torch.cuda.empty_cache()


def test_plan_persistent_equatorial_benchmark_box(oz):
    """The benchmark's equatorial workload: the z >= 0 half (256 x 256 x 128
    cells) of the 256^3 puncture box, reflection at z = 0 and Sommerfeld
    elsewhere, in a persistent plan (8x8x8 bricks, two waves), one RK4 step
    replayed from the graph.  Stages 3 and 4 against the oracle at sampled
    points (the plane's layers among them); the step bitwise equal to the
    non-persistent single-box path."""
    print("case: persistent plan, equatorial half of the 256^3 punctures", flush=True)
    g, u, dt = I.config_punctures_equatorial(256)
    ozp = _ozp(oz, z4c.default_params())
    plan = z4c.Plan([I.Box(g, u, None, dt)], tile=PERSISTENT)
    plan.step(1, use_graph=True)
    a, b, acc, _ = plan._keep[0]
    new, a_h, b_h, acc_h = to_host(plan.u[0]), to_host(a), to_host(b), to_host(acc)
    plan.close()
    del plan, a, b, acc
    torch.cuda.empty_cache()
    ng = g.ng
    pts = evolved_points(g, sample=3000, seed=3)
    plane = np.array([(i, j, k) for i in (ng, 64, 200, g.n[0] + ng - 1) for j in (ng, 128, g.n[1] + ng - 1)
                      for k in (ng, ng + 1, ng + 2)], dtype=pts.dtype)
    pts = np.concatenate([pts, plane])
    check_stage(oz, ozp, g, 3, dt, b_h, u, None, a_h, None, pts, "equatorial plan")
    check_stage(oz, ozp, g, 4, dt, a_h, None, acc_h, new, None, pts, "equatorial plan")
    del a_h, b_h, acc_h
    st = z4c.Stepper(g, u, dt)  # default tile: not persistent
    st.step(1)
    got = to_host(st.u)
    # the plan leaves the mirrored layers to the next step's fill; compare
    # what both paths evolve
    m = np.zeros(g.shape[1:], dtype=bool)
    m[ng:] = True
    assert np.array_equal(got[:, m], new[:, m])
    del st
    torch.cuda.empty_cache()


def test_plan_graph_stages_three_boxes(oz):
    """Three copy boxes of uneven size in one plan, graph replays: stages 3
    and 4 of every box at every step against the oracle (all active points)."""
    print("case: plan of 3 copy boxes (20^3, 16^3, 12^3), graph, 2 steps, stages 3 and 4", flush=True)
    boxes = I.config_hierarchy(sizes=(20, 16, 12))
    ozp = _ozp(oz, z4c.default_params())
    plan = z4c.Plan(boxes, tile=PERSISTENT)
    for step in range(2):
        old = [to_host(x) for x in plan.u]
        plan.step(1, use_graph=True)
        for bx, un, ub, keep in zip(boxes, old, plan.u, plan._keep):
            a, b, acc, _ = keep
            pts = evolved_points(bx.grid)
            lab = f"plan box {bx.grid.n[0]}^3 step {step}"
            check_stage(oz, ozp, bx.grid, 3, bx.dt, to_host(b), un, None, to_host(a), None, pts, lab)
            check_stage(oz, ozp, bx.grid, 4, bx.dt, to_host(a), None, to_host(acc), to_host(ub), None, pts, lab)
    plan.close()


def test_plan_nine_boxes_benchmark_sizes(oz):
    """The benchmark's 9-box workload (copy boxes of 160^3 down to 64^3, 13.5 M
    active cells) in one persistent plan (8x8x8 bricks, two waves), one step
    replayed from the graph: stages 3 and 4 of every box against the oracle
    at sampled points."""
    print("case: plan of the 9 benchmark boxes (160^3 .. 64^3), persistent, graph, stages 3 and 4", flush=True)
    boxes = I.config_hierarchy()
    ozp = _ozp(oz, z4c.default_params())
    old = [bx.state for bx in boxes]
    plan = z4c.Plan(boxes, tile=PERSISTENT)
    plan.step(1, use_graph=True)
    for k, (bx, un, ub, keep) in enumerate(zip(boxes, old, plan.u, plan._keep)):
        a, b, acc, _ = keep
        pts = evolved_points(bx.grid, sample=600, seed=k)
        lab = f"plan box {bx.grid.n[0]}^3"
        check_stage(oz, ozp, bx.grid, 3, bx.dt, to_host(b), un, None, to_host(a), None, pts, lab)
        check_stage(oz, ozp, bx.grid, 4, bx.dt, to_host(a), None, to_host(acc), to_host(ub), None, pts, lab)
    plan.close()
    torch.cuda.empty_cache()


def _covered(gp, children):
    """Active-cell mask of parent grid gp with the cells that a child
    (grid, F) covers removed (those are overwritten by restriction)."""
    m = gp.active_mask()
    ng = gp.ng
    for gc, F in children:
        lo = [ng + F[d] for d in range(3)]
        hi = [lo[d] + gc.n[d] // 2 for d in range(3)]
        m[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = False
    return m


def _mask_points(m, sample=None, seed=0):
    kk, jj, ii = np.nonzero(m)
    pts = np.stack([ii, jj, kk], axis=1).astype(np.int32)
    if sample is not None and sample < len(pts):
        pts = pts[np.random.default_rng(seed).choice(len(pts), sample, replace=False)]
    return pts


def test_hierarchy_stage4_prolonged_ghosts(oz):
    """Three levels of 24^3 (Sommerfeld root): after a root step, the last
    stage of each level's last step is checked on the level's own buffers
    (A = u3 with the ghosts the GPU filled -- prolonged and interpolated in
    time for levels 1 and 2 --, acc = acc3) at every cell that restriction
    did not overwrite afterwards, and on the root's evolved ghosts."""
    print("case: hierarchy 3 x 24^3, stage 4 with prolonged ghosts vs oracle", flush=True)
    levels = []
    for g, F in I.bo_level_grids(3, 24, 1.0):
        uu = I.brill_lindquist_state(g) + 1e-3 * (I.random_strong_field_state(g, seed=3) - I.flat_state(g))
        levels.append((g, I.pi_symmetrize(uu), F))
    dt0 = 0.5 * levels[0][0].h[0]
    ozp = _ozp(oz, z4c.default_params())
    H = z4c.Hierarchy(levels, dt0)
    H.advance(2, use_graph=True)
    for q, (g, _, F) in enumerate(levels):
        a, b, acc = H._keep[q][0], H._keep[q][1], H._keep[q][2]
        m = _covered(g, [(levels[q + 1][0], levels[q + 1][2])] if q + 1 < len(levels) else [])
        if q == 0:
            m = m | ~g.active_mask()  # the root's Sommerfeld ghosts are evolved
        pts = _mask_points(m)
        dt = dt0 / 2 ** q
        check_stage(oz, ozp, g, 4, dt, to_host(a), None, to_host(acc), to_host(H.u[q]), None, pts,
                    f"hierarchy level {q}")
    H.close()


def test_hierarchy_bbh_persistent_bitwise_and_stage4(oz):
    """Binary-black-hole layout (128^3 root and fixed levels, moving 64^3
    pairs): one root step with the default persistent launch is bitwise equal
    to the non-persistent launch; the deepest fixed 128^3 level's last stage
    is checked against the oracle at sampled cells outside its children."""
    print("case: BBH hierarchy persistent vs non-persistent, stage 4 of a 128^3 level", flush=True)
    pt, states, dt0, xp = I.config_bbh_moving()
    lv = [(g, u, F, par, obj) for (g, F, par, obj), u in zip(pt, states)]
    out = []
    ozp = _ozp(oz, z4c.default_params())
    for tile in (None, z4c.Tile(8, 8, 8, 2, 0)):
        H = z4c.Hierarchy(lv, dt0, tile=tile)
        H.set_moving(xp)
        H.advance(1)
        out.append([to_host(x) for x in H.u])
        if tile is None:
            q = 3  # deepest fixed level (128^3, h = 0.25); its children are the two moving 64^3 patches
            g = pt[q][0]
            kids = [(pt[c][0], pt[c][1]) for c in range(len(pt)) if pt[c][2] == q]
            pts = _mask_points(_covered(g, kids), sample=3000, seed=3)
            a, acc = H._keep[q][0], H._keep[q][2]
            check_stage(oz, ozp, g, 4, dt0 / 2 ** q, to_host(a), None, to_host(acc), out[0][q], None, pts,
                        "bbh level 3 (128^3)")
            del a, acc
        H.close()
        del H
        torch.cuda.empty_cache()
    for p, (x, y) in enumerate(zip(*out)):
        assert np.array_equal(x, y), p
