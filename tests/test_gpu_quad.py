"""Multi-point triangle quadrature of the exact path (TPE_OPT_QUADRATURE) against the oracle's."""
import contextlib

import numpy as np
import pytest

import oracle
from paper_2509_22110_amd import meshes as M
from tests.gpu_util import log, needs_gpu, rel_energy, rel_grad_maxnorm, tpe, upload

pytestmark = [pytest.mark.gpu, needs_gpu]
E_TOL, G_TOL = 1e-6, 1e-5


@contextlib.contextmanager
def quadrature(T, dev, Q):
    ctx = T.context(dev)
    ctx.set_option(T.OPT_QUADRATURE, Q)
    try:
        yield ctx
    finally:
        ctx.set_option(T.OPT_QUADRATURE, 1)


def meshes():
    X, F = M.icosphere(1)
    yield "L1-jitter", M.radial_jitter(X, 0.02, 1), F
    X2, F2 = M.icosphere(2)
    Xb, _, _ = M.bump(X2, 0, 0.3, 0.1)
    yield "L2-bump", Xb, F2
    c = M.make_config("C1")
    yield "C1", c.X, c.F


@pytest.mark.parametrize("Q", [3, 6])
@pytest.mark.parametrize("name,X,F", list(meshes()), ids=lambda v: v if isinstance(v, str) else "")
def test_parity(Q, name, X, F):
    T = tpe()
    Xd, Fd = upload(X, F)
    with quadrature(T, Xd.device, Q):
        E, G = T.gradient(Xd, Fd)
        Ee = T.energy(Xd, Fd)
    Eo, Go = oracle.gradient_quad(X, F, Q)
    eE, eEe, eG = rel_energy(float(E.cpu()), Eo), rel_energy(float(Ee.cpu()), Eo), rel_grad_maxnorm(G.cpu().numpy(), Go)
    log(name, "Q", Q, "rel E", eE, "rel E(energy kernel)", eEe, "rel G", eG)
    assert eE <= E_TOL and eEe <= E_TOL and eG <= G_TOL


def test_level4_six_points():
    """5,120 faces x 36 point pairs per face pair (9.4e8 point pairs)."""
    T = tpe()
    X, F = M.icosphere(4)
    X, _ = M.sh_deform(X, 2, 8, 0.05, 3)
    Xd, Fd = upload(X, F)
    with quadrature(T, Xd.device, 6):
        E, G = T.gradient(Xd, Fd)
    log("L4 six-point oracle start")
    Eo, Go = oracle.gradient_quad(X, F, 6)
    eE, eG = rel_energy(float(E.cpu()), Eo), rel_grad_maxnorm(G.cpu().numpy(), Go)
    log("L4 Q 6 rel E", eE, "rel G", eG)
    assert eE <= E_TOL and eG <= G_TOL


def test_one_point_option_is_the_default_path():
    T = tpe()
    c = M.make_config("C1")
    Xd, Fd = upload(c.X, c.F)
    E0, G0 = T.gradient(Xd, Fd)
    with quadrature(T, Xd.device, 1):
        E1, G1 = T.gradient(Xd, Fd)
    assert float(E0.cpu()) == float(E1.cpu()) and np.array_equal(G0.cpu().numpy(), G1.cpu().numpy())


def test_rules_differ_and_errors():
    T = tpe()
    c = M.make_config("C1")
    Xd, Fd = upload(c.X, c.F)
    E1 = float(T.energy(Xd, Fd).cpu())
    with quadrature(T, Xd.device, 6):
        E6 = float(T.energy(Xd, Fd).cpu())
        tree = T.build_tree(Xd, Fd)
        with pytest.raises(T.TPEError):  # the far field is one point per face
            T.farfield(tree, Xd, Fd)
        with pytest.raises(T.TPEError):  # and so is the confinement energy
            T.conf_energy(Xd, Fd, 1.2 * Xd, Fd)
    assert abs(E6 - E1) > 1e-4 * E1  # a different rule is a different discretisation
    ctx = T.context(Xd.device)
    with pytest.raises(T.TPEError):
        ctx.set_option(T.OPT_QUADRATURE, 2)
