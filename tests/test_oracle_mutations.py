"""Plant plausible mistakes in the oracle (CPU only) and check that the pins
catch every one of them.

Each mutation edits one line of the oracle's source text, loads the edited
module under a private name and runs the pin suite against it; the test
passes when at least one pin fails. Together with ``test_oracle_pins.py``
this shows the pins pin the oracle: the correct oracle passes them all, and a
dropped term, a wrong sign or index, or a transposed operand does not.
"""
import importlib.util
import os
import sys
import types

import pytest

import pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = [
    ("graph64", "return np.sqrt((Li * Li).sum(axis=0))", "return np.sqrt((Li * Li).sum(axis=1))",
     "row norms of L^-1 instead of column norms in the image bound"),
    ("graph64", "    v = f @ L\n", "    v = f @ L.T\n", "column-vector lattice convention"),
    ("graph64", "d = x - x[i]", "d = x[i] - x", "displacement sign x_i - x_j"),
    ("graph64", "keep[i, self_t[0]] = False", "pass", "self-image (i, i, 0) kept"),
    ("graph64", "m = length < R", "m = length <= R", "non-strict cutoff"),
    ("graph64", "R = float(radii[int(i)]) + float(band)", "R = float(radii.max()) + float(band)",
     "largest per-atom cutoff used for every source"),
    ("graph64", "lo = np.ceil(-R * r - d - _BOX_SLACK)", "lo = np.ceil(-R * r + d - _BOX_SLACK)",
     "sign error in the lower image bound"),
    ("graph64", "hi = np.floor(R * r - d + _BOX_SLACK)", "hi = np.floor(R * r - d + _BOX_SLACK - 1)",
     "off-by-one upper image bound"),
    ("graph64", "order = np.lexsort((t[:, 2], t[:, 1], t[:, 0], j, ln))",
     "order = np.lexsort((t[:, 0], t[:, 1], t[:, 2], j, ln))", "KNN ties ordered by reversed t"),
    ("graph64", "order = np.lexsort((t[:, 2], t[:, 1], t[:, 0], j, ln))",
     "order = np.lexsort((t[:, 2], t[:, 1], t[:, 0], ln, j))", "KNN ordered by dst before length"),
    ("graph64", "sel = order[:k]", "sel = order[1:k + 1]", "KNN off-by-one selection"),
    ("graph64", "keep = ln <= dk[r]", "keep = ln < dk[r]", "ties at the k-th distance dropped"),
    ("symmetrize64", "out_img.append(-img[e])", "out_img.append(img[e])", "reverse edge keeps +t"),
    ("symmetrize64", "if (j, i, -int(t[0]), -int(t[1]), -int(t[2])) not in present:",
     "if (j, i, int(t[0]), int(t[1]), int(t[2])) not in present:", "presence test on (j, i, +t)"),
    ("triplets64", "keep = a != b", "keep = a >= 0", "triplets include the pair (g, g)"),
    ("triplets64", "b = np.tile(idx, d)", "b = np.repeat(idx, d)", "second edge of the pair not varied"),
    ("triplets64", "den = np.sqrt((a * a).sum(1)) * np.sqrt((b * b).sum(1))", "den = (a * a).sum(1)",
     "angle normalised by the first edge's squared length"),
    ("geometry64", "+ np.asarray(image, np.float64)", "+ 0.0 * np.asarray(image, np.float64)",
     "image offset dropped from the edge vector"),
    ("geometry64", 'v = np.einsum("ek,ekm->em", f, lattices[s])', 'v = np.einsum("ek,emk->em", f, lattices[s])',
     "transposed lattice in the edge vector"),
    ("geometry64", 'gx = np.einsum("em,ekm->ek", g, Ls)', 'gx = np.einsum("em,emk->ek", g, Ls)',
     "g L instead of g L^T in the coordinate gradient"),
    ("geometry64", "np.add.at(grad_frac, src, -gx)", "np.add.at(grad_frac, src, gx)",
     "wrong sign of the source-atom gradient"),
    ("geometry64", "np.add.at(grad_frac, src, -gx)", "pass", "source-atom gradient dropped"),
    ("geometry64", "f[:, :, None] * g[:, None, :]", "g[:, :, None] * f[:, None, :]",
     "transposed lattice gradient"),
    ("geometry64", "gl / safe, 0.0)", "gl, 0.0)", "length gradient not divided by the length"),
    ("geometry64", "return -2.0 * w * (length - mu)", "return 2.0 * w * (length - mu)",
     "wrong sign of the loss gradient"),
    ("geometry64", "return -2.0 * w * (length - mu)", "return -1.0 * w * (length - mu)",
     "factor 2 of the loss gradient dropped"),
    ("geometry64", "np.exp(-(length - mu) ** 2)).sum()", "np.exp(-(length - mu))).sum()",
     "square dropped from the loss exponent"),
]


def _load_mutated(module, old, new):
    path = os.path.join(ROOT, "oracle", module + ".py")
    with open(path) as f:
        src = f.read()
    assert src.count(old) == 1, (module, old)
    name = "_mutated_oracle_" + module
    spec = importlib.util.spec_from_loader(name, loader=None)
    mod = importlib.util.module_from_spec(spec)
    sys.modules[name] = mod          # dataclasses look their module up here
    try:
        exec(compile(src.replace(old, new), path + " (mutated)", "exec"), mod.__dict__)
    finally:
        del sys.modules[name]
    return mod


def _oracle_with(module, old, new):
    import oracle
    ns = types.SimpleNamespace(**{k: getattr(oracle, k) for k in oracle.__all__})
    mod = _load_mutated(module, old, new)
    for k in oracle.__all__:
        if hasattr(mod, k):
            setattr(ns, k, getattr(mod, k))
    return ns


@pytest.mark.parametrize("module,old,new,desc", MUTATIONS, ids=[m[3] for m in MUTATIONS])
def test_mutation_is_caught(module, old, new, desc):
    O = _oracle_with(module, old, new)
    for pin in pins.ALL_PINS:
        try:
            pin(O)
        except Exception:
            return
    pytest.fail("no pin caught the planted mistake: " + desc)
