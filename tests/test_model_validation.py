"""Model validation of ms_model_create (host logic, no GPU needed: every
check runs before the first device call). Each case breaks one property of a
valid synthetic model and expects the documented status code; the valid
models themselves are created on the GPU by the parity tests."""
import numpy as np
import pytest

from paper_2603_29332_amd import ms, synth

E_MODEL, E_UNSUPPORTED = -4, -5


def _chain():
    return {k: (np.array(v) if isinstance(v, np.ndarray) else v)
            for k, v in synth.chain_model(1).items()}


def _drop_via(m, k):
    """Muscle k's path without its last via-point."""
    vs = m["via_start"].copy()
    cut = vs[k + 1] - 1
    m["via_node"] = np.delete(m["via_node"], cut)
    m["via_pos"] = np.delete(m["via_pos"], cut, axis=0)
    vs[k + 1:] -= 1
    m["via_start"] = vs
    return m


def _extra_vias(m, k, n):
    """Muscle k's path with n more via-points on its origin's body."""
    vs = m["via_start"].copy()
    at = vs[k] + 1
    m["via_node"] = np.insert(m["via_node"], at, [m["via_node"][vs[k]]] * n)
    m["via_pos"] = np.insert(m["via_pos"], at, [m["via_pos"][vs[k]] + 0.01] * n, axis=0)
    vs[k + 1:] += n
    m["via_start"] = vs
    return m


def _tiled_muscles(m, reps):
    """The chain's muscles repeated reps times."""
    nm, vs = m["n_mus"], m["via_start"]
    for k in ("f0", "l_opt", "l_slack", "v_max", "tau_act", "tau_deact"):
        m[k] = np.tile(m[k], reps)
    nv = vs[-1]
    m["via_start"] = np.concatenate([vs[:-1] + r * nv for r in range(reps)] + [[reps * nv]])
    m["via_node"] = np.tile(m["via_node"], reps)
    m["via_pos"] = np.tile(m["via_pos"], (reps, 1))
    m["n_mus"] = nm * reps
    return m


def _set(name, idx, value):
    def f(m):
        a = m[name].copy()
        a[idx] = value
        m[name] = a
        return m
    return f


CASES = {
    "parent after child": (_set("parent", 3, 5), E_MODEL, "parent"),
    "unknown joint type": (_set("jtype", 2, 3), E_MODEL, "jtype"),
    "free joint below the root": (_set("jtype", 4, 2), E_MODEL, "free joint"),
    "axis not unit": (_set("axis", (2, 0), 3.0), E_MODEL, "unit"),
    "negative mass": (_set("mass", 1, -1.0), E_MODEL, ""),
    "pose box inverted": (lambda m: _set("qlo", 0, 1.0)(_set("qhi", 0, -1.0)(m)), E_MODEL, "qlo"),
    "negative damping": (_set("damping", 0, -0.1), E_MODEL, "damping"),
    "one via-point": (lambda m: _drop_via(m, 0), E_MODEL, "2 via-points"),
    "nine via-points": (lambda m: _extra_vias(m, 0, 7), E_UNSUPPORTED, "8 via-points"),
    "via node out of range": (_set("via_node", 1, 99), E_MODEL, "via_node"),
    "zero optimal fibre length": (_set("l_opt", 3, 0.0), E_MODEL, "Hill"),
    "more than 1024 muscles": (lambda m: _tiled_muscles(m, 65), E_UNSUPPORTED, "n_mus"),
}


@pytest.mark.parametrize("case", list(CASES))
def test_invalid_model_is_rejected(case):
    edit, code, text = CASES[case]
    m = edit(_chain())
    with pytest.raises(ms.MsError) as ei:
        ms.Model(m)
    assert ei.value.code == code
    assert text in str(ei.value)


def test_contact_checks():
    m = synth.human_model(2)
    for key, idx, value, text in (("con_node", 0, 500, "con_node"),
                                  ("con_radius", 1, -0.01, "radius")):
        b = dict(m)
        b[key] = np.array(m[key]).copy()
        b[key][idx] = value
        with pytest.raises(ms.MsError) as ei:
            ms.Model(b)
        assert ei.value.code == E_MODEL and text in str(ei.value)


def _coupled(dofs_coefs, k=100.0, d=1.0, base=None):
    """A model with one joint-coupling constraint per entry of dofs_coefs
    (a list of [(dof, coef), ...])."""
    m = dict(base if base is not None else _chain())
    start, dofs, coefs = [0], [], []
    for terms in dofs_coefs:
        for j, c in terms:
            dofs.append(j)
            coefs.append(c)
        start.append(len(dofs))
    m["n_eq"] = len(start) - 1
    m["eq_start"] = np.array(start, np.int32)
    m["eq_dof"] = np.array(dofs, np.int32)
    m["eq_coef"] = np.array(coefs, np.float32)
    m["eq_off"] = np.zeros(len(start) - 1, np.float32)
    m["eq_k"], m["eq_d"] = np.float32(k), np.float32(d)
    return m


COUPLING_CASES = {
    "duplicate DoF in a constraint": ([[(2, 1.0), (2, -0.5)]], {}, E_MODEL, "twice"),
    "DoF out of range": ([[(2, 1.0), (9, -0.5)]], {}, E_MODEL, "eq_dof"),
    "nine terms": ([[(j % 8, 1.0) for j in range(9)]], {}, E_MODEL, "1 to 8 terms"),
    "negative stiffness": ([[(2, 1.0), (5, -0.5)]], {"k": -1.0}, E_MODEL, "eq_k"),
    "more constraints than DoFs": ([[(j, 1.0)] for j in range(8)] + [[(0, 2.0)]], {}, E_MODEL,
                                   "more constraints"),
}


@pytest.mark.parametrize("case", list(COUPLING_CASES))
def test_invalid_coupling_is_rejected(case):
    terms, kw, code, text = COUPLING_CASES[case]
    with pytest.raises(ms.MsError) as ei:
        ms.Model(_coupled(terms, **kw))
    assert ei.value.code == code
    assert text in str(ei.value)


def test_coupling_needs_one_path_and_hinge_dofs():
    """On the whole body: DoFs of the two arms are not on one root-to-leaf
    path (the matrix would lose its tree sparsity), and a free root's DoFs
    cannot be coupled."""
    m = synth.human_model(2)
    lab = m["node_label"]
    dof, k = {}, 0
    for i, t in enumerate(m["jtype"]):
        dof[lab[i]] = k
        k += 6 if t == 2 else 1
    for terms, text in (([[(dof["humL:2"], 1.0), (dof["humR:2"], -1.0)]], "one root-to-leaf path"),
                        ([[(2, 1.0), (dof["humL:2"], -1.0)]], "hinge/slide DoF")):
        with pytest.raises(ms.MsError) as ei:
            ms.Model(_coupled(terms, base=m))
        assert ei.value.code == E_MODEL and text in str(ei.value)
