"""Helpers shared by the GPU tests: device placement of seeded inputs."""
import numpy as np
import torch

DEV = torch.device("cuda", 0)


def t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def scene_tensors(s):
    return [t(a) for a in s.arrays()]


def log(msg):
    print(msg, flush=True)


def grad_close(got, want, name, want_abs=None, rel=1e-3, floor=1e-2, kappa=1e-5):
    """Element-wise gradient bar, no exceptions:
        |g - g_ref| <= max(rel * max(|g_ref|, floor * max|g_ref|), kappa * S)
    where S (want_abs, from the oracle) is the element's error scale: the
    magnitudes of its per-hit terms plus the chain rule applied to the
    magnitudes of the sums each hit's dL/dalpha is formed from.  A
    single-precision evaluation errs by a few ulps (6e-8) of what it adds and
    subtracts, so by about 1e-6 S; kappa = 1e-5 leaves a factor 10.  Also
    the block's relative L2 error <= rel."""
    import numpy as np
    got = np.asarray(got, np.float64).reshape(want.shape)
    scale = np.abs(want).max()
    if scale == 0:
        assert np.abs(got).max() == 0, name
        return
    base = rel * np.maximum(np.abs(want), floor * scale)
    tol = base if want_abs is None else np.maximum(base, kappa * want_abs.reshape(want.shape))
    err = np.abs(got - want)
    bad = err > tol
    l2 = np.linalg.norm(got - want) / np.linalg.norm(want)
    over = err > base
    via_s = (f", {int(over.sum())} past the relative bar, worst of them err/(kappa S) "
             f"{float((err[over] / tol[over]).max()):.3g}") if over.any() else ""
    print(f"  grads {name}: bad {int(bad.sum())} of {bad.size}, worst err/tol {float((err / tol).max()):.3g}"
          f"{via_s}, rel L2 {l2:.3g}", flush=True)
    assert not bad.any(), (name, int(bad.sum()), float((err / tol).max()), scale)
    assert l2 < rel, (name, l2)
