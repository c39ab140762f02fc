"""Tiny hand-built models for the oracle's closed-form pins."""
import numpy as np

from paper_2603_29332_amd import synth


def _base(parent, jtype, jpos, axis, mass, com, inertia, damping=None,
          muscles=(), contacts=(), contact=(1e5, 1e3, 1.0, 0.2),
          gravity=(0, 0, -9.81)):
    n = len(parent)
    nv = sum(6 if t == 2 else 1 for t in jtype)
    f0, lo, ls, vn, vp, vs = [], [], [], [], [], [0]
    for (F0, lopt, lsl, pts) in muscles:
        f0.append(F0)
        lo.append(lopt)
        ls.append(lsl)
        for nd, p in pts:
            vn.append(nd)
            vp.append(p)
        vs.append(len(vn))
    nm = len(f0)
    model = dict(
        name="tiny", parent=parent, jtype=jtype, jpos=jpos,
        jrot=np.tile(np.eye(3).ravel(), (n, 1)), axis=axis, mass=mass, com=com,
        inertia=inertia,
        damping=np.zeros(nv) if damping is None else damping,
        qlo=np.full(nv, -np.pi), qhi=np.full(nv, np.pi),
        f0=f0, l_opt=lo, l_slack=ls, v_max=np.full(nm, 10.0),
        tau_act=np.full(nm, 0.010), tau_deact=np.full(nm, 0.040),
        via_start=vs, via_node=vn, via_pos=np.array(vp).reshape(-1, 3),
        con_node=[c[0] for c in contacts],
        con_pos=np.array([c[1] for c in contacts]).reshape(-1, 3),
        con_radius=[c[2] for c in contacts], contact=list(contact),
        gravity=list(gravity))
    return synth._finish(model)


def pendulum(m=2.0, d=0.4, Ic=0.01, damping=0.0, muscles=()):
    """One hinge about y at the origin; COM at distance d along -z."""
    return _base([-1], [0], [[0, 0, 0]], [[0, 1, 0]], [m], [[0, 0, -d]],
                 [[Ic, Ic, Ic]], damping=[damping], muscles=muscles)


def two_link(m1=1.5, m2=0.8, l1=0.5, lc1=0.25, lc2=0.2, I1=0.03, I2=0.01):
    """Planar 2-link arm, both hinges about y, links along -z at q = 0."""
    return _base([-1, 0], [0, 0], [[0, 0, 0], [0, 0, -l1]],
                 [[0, 1, 0], [0, 1, 0]], [m1, m2],
                 [[0, 0, -lc1], [0, 0, -lc2]], [[I1, I1, I1], [I2, I2, I2]])


def point_mass_slides(m=1.5, radius=0.02, contact=(1e5, 1e3, 1.0, 0.2)):
    """Three slides (x, y, z) carrying a point mass with one sphere."""
    return _base([-1, 0, 1], [1, 1, 1], [[0, 0, 0]] * 3,
                 [[1, 0, 0], [0, 1, 0], [0, 0, 1]], [0, 0, m],
                 [[0, 0, 0]] * 3, [[0, 0, 0], [0, 0, 0], [1e-4] * 3],
                 contacts=[(2, [0, 0, 0], radius)], contact=contact)


def free_body(m=3.0, inertia=(0.02, 0.05, 0.08), com=(0.0, 0.0, 0.0),
              gravity=(0, 0, -9.81)):
    """A single free-floating rigid body."""
    return _base([-1], [2], [[0, 0, 0]], [[0, 0, 0]], [m], [list(com)],
                 [list(inertia)], gravity=gravity)


def mixed_chain():
    """Fixed base 1.015 m up; hinge y, slide z, hinge x, slide x, hinge y down
    a 1 m chain; a tip sphere just touching the ground; five muscles spanning
    hinges and slides (one or two joints each), tendon slacks set so that the
    fibres sit at their optimal length at q = 0."""
    from oracle import Oracle
    parent = [-1, 0, 1, 2, 3]
    jtype = [0, 1, 0, 1, 0]
    jpos = [[0, 0, 1.015], [0, 0, -0.3], [0, 0, -0.1], [0, 0, -0.3], [0.05, 0, -0.1]]
    axis = [[0, 1, 0], [0, 0, 1], [1, 0, 0], [1, 0, 0], [0, 1, 0]]
    mass = [2.0, 1.0, 1.5, 0.8, 0.6]
    com = [[0, 0, -0.15], [0, 0, -0.05], [0, 0, -0.15], [0, 0, -0.05], [0, 0, -0.1]]
    inertia = [[0.02, 0.02, 0.005], [0.005] * 3, [0.01, 0.01, 0.003], [0.003] * 3, [0.002] * 3]
    mus = [(800.0, 0.10, 0.0, [(-1, [0.03, 0, 0.97]), (0, [0.03, 0, -0.2])]),
           (600.0, 0.08, 0.0, [(0, [0.02, 0.02, -0.1]), (1, [0.02, 0, -0.05])]),
           (700.0, 0.12, 0.0, [(1, [0, 0.03, -0.02]), (2, [0, 0.03, -0.1]), (3, [0, 0.02, -0.05])]),
           (500.0, 0.09, 0.0, [(2, [-0.03, 0, -0.05]), (4, [-0.02, 0, -0.05])]),
           (900.0, 0.11, 0.0, [(-1, [-0.03, 0, 0.97]), (1, [-0.03, 0, -0.02])])]
    m = _base(parent, jtype, jpos, axis, mass, com, inertia, damping=[0.1] * 5,
              muscles=mus, contacts=[(4, [0, 0, -0.2], 0.02)])
    L0 = Oracle(m).geometry(np.zeros(m["nq"]), np.zeros(m["nv"]))[0]
    m["l_slack"] = (L0 - m["l_opt"]).astype(m["l_slack"].dtype)
    return m


def twin_chains(n_link=6, seed=4):
    """Two equal fixed-base hinge chains on separate roots, the second a copy
    of the first 0.5 m to the side and without muscles: the top height level
    of the DoF tree holds two rows."""
    m = synth.chain_model(seed, n_link=n_link, n_mus=12)
    n = n_link
    two = dict(m)
    two["parent"] = np.concatenate([m["parent"], np.where(m["parent"] >= 0, m["parent"] + n, -1)])
    jpos2 = np.array(m["jpos"]).copy()
    jpos2[0, 0] += 0.5
    two["jpos"] = np.concatenate([m["jpos"], jpos2])
    for k in ("jtype", "jrot", "axis", "mass", "com", "inertia", "damping", "qlo", "qhi"):
        two[k] = np.concatenate([m[k], m[k]])
    two["name"] = f"twin{n}"
    return synth._finish(two)


def maxwell_slide(m=2.0, F0=500.0, l_opt=0.1, l_slack=0.2, d=0.28):
    """A point mass on a slide along x with one muscle from the world point
    (-d, 0, 0) to the mass: path length L = d + x, moment arm -1. No
    gravity, no damping."""
    return _base([-1], [1], [[0, 0, 0]], [[1, 0, 0]], [m], [[0, 0, 0]], [[1e-4] * 3],
                 muscles=[(F0, l_opt, l_slack, [(-1, [-d, 0, 0]), (0, [0, 0, 0])])],
                 gravity=(0, 0, 0))


def fixed_path_muscle(F0=800.0, l_opt=0.1, l_slack=0.2, L=0.31):
    """A muscle whose path (length L) runs between two world points beside a
    slide that it does not cross."""
    return _base([-1], [1], [[0, 0, 0]], [[1, 0, 0]], [1.0], [[0, 0, 0]], [[1e-4] * 3],
                 muscles=[(F0, l_opt, l_slack, [(-1, [0, 1, 0]), (-1, [L, 1, 0])])],
                 gravity=(0, 0, 0))
