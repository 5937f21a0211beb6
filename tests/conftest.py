import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def tiny_pack():
    """A small trained model pack (12x8 grid, 2x2 subdomains) built by the oracle."""
    from oracle.build_model import build
    pack, X, mus, _ = build("tiny", workers=1, verbose=False)
    return pack


@pytest.fixture(scope="session")
def cfg0_pack():
    """The 36x36, 2x2 workload's model pack, built by the oracle pipeline (seconds)."""
    import numpy as np
    path = os.path.join(ROOT, "models", "cfg0.npz")
    if os.path.exists(path):
        return dict(np.load(path, allow_pickle=False))
    from oracle.build_model import build
    pack, *_ = build("cfg0", workers=1, verbose=False)
    return pack


@pytest.fixture(scope="session")
def tinymix_pack():
    """16x12 grid, 2x2 subdomains whose latent sizes (from {4, 6, 8, 12}) and hyper-reduction
    fractions (0.3 to 0.6) differ per subdomain."""
    from oracle.build_model import build
    pack, *_ = build("tinymix", workers=1, verbose=False)
    return pack


@pytest.fixture(scope="session")
def tinywide_pack():
    """40x8 grid, 2x2 subdomains, Swish, band-5 shift-5 masks (window 55 hidden units: the
    decoder's wide ring), latents (8, 4)."""
    from oracle.build_model import build
    pack, *_ = build("tinywide", workers=1, verbose=False)
    return pack


@pytest.fixture(scope="session")
def tinyl10_pack():
    """40x8, 2x2, Swish band-5 shift-5 masks, latents (10, 5)."""
    from oracle.build_model import build
    pack, *_ = build("tinyl10", workers=1, verbose=False)
    return pack


@pytest.fixture(scope="session")
def tinyl16_pack():
    """40x8, 2x2, Swish band-5 shift-5 masks, latents (16, 8): 24 latents per subdomain."""
    from oracle.build_model import build
    pack, *_ = build("tinyl16", workers=1, verbose=False)
    return pack


@pytest.fixture(scope="session")
def tinybig_pack():
    """48x48 grid, 8x8 subdomains, 96 constraints: the KKT system exceeds one wave's rows."""
    from oracle.build_model import build
    pack, *_ = build("tinybig", workers=1, verbose=False)
    return pack


@pytest.fixture(scope="session")
def tinyhuge_pack():
    """48x48 grid, 8x8 subdomains, latents (12, 6), 192 constraints: the Schur system exceeds
    the LDS a workgroup holds."""
    from oracle.build_model import build
    pack, *_ = build("tinyhuge", workers=1, verbose=False)
    return pack


@pytest.fixture(scope="session")
def headline_pack():
    """The 240x240, 4x4, latent (8,4) workload's model pack: the trained pack the benchmark
    solves (models/cfg1.npz, written by the oracle pipeline) when present, else a pack of the
    same shape built by the oracle pipeline at a small training budget (about a minute)."""
    import numpy as np
    path = os.path.join(ROOT, "models", "cfg1.npz")
    if os.path.exists(path):
        return "cfg1", dict(np.load(path, allow_pickle=False))
    from oracle.build_model import build
    pack, *_ = build("cfg1shape", workers=min(4, os.cpu_count() or 1), verbose=False)
    return "cfg1shape", pack


@pytest.fixture(scope="session")
def tinysrpc2x1_pack():
    """16x8 grid, 2x1 split, strong ROM-port constraint: one port of 3-band port decoders
    ((b, s) = (3, 3), sigmoid), latents (4, 2)."""
    from oracle.build_model import build
    pack, *_ = build("tinysrpc2x1", workers=1, verbose=False)
    return pack


@pytest.fixture(scope="session")
def tinysrpc3x1_pack():
    """24x8 grid, 3x1 split, strong ROM-port constraint: the middle subdomain carries two
    ports (latents (4, 4)), the outer ones one (latents (4, 2))."""
    from oracle.build_model import build
    pack, *_ = build("tinysrpc3x1", workers=1, verbose=False)
    return pack


@pytest.fixture(scope="session")
def tinyls_pack():
    """LS-ROM on the 12x8, 2x2 split: POD bases (latents (4, 2)) with the tiny model's HR nodes."""
    from oracle.build_model import build
    pack, *_ = build("tinyls", workers=1, verbose=False)
    return pack


@pytest.fixture(scope="session")
def tinylsg_pack():
    """tinyls with gappy-POD HR: B_i = (Z_i Phi_i^r)^+ Z_i on the same nodes."""
    from oracle.build_model import build
    pack, *_ = build("tinylsg", workers=1, verbose=False)
    return pack


@pytest.fixture(scope="session")
def cfg0lsg_pack():
    """cfg0ls with gappy-POD HR on the same nodes."""
    from oracle.build_model import build
    pack, *_ = build("cfg0lsg", workers=1, verbose=False)
    return pack


@pytest.fixture(scope="session")
def cfg0ls_pack():
    """LS-ROM of the 36x36, 2x2 workload: POD bases (6, 3), the same HR nodes and C as its
    nonlinear-manifold model."""
    import numpy as np
    path = os.path.join(ROOT, "models", "cfg0ls.npz")
    if os.path.exists(path):
        return dict(np.load(path, allow_pickle=False))
    from oracle.build_model import build
    pack, *_ = build("cfg0ls", workers=1, verbose=False)
    return pack
