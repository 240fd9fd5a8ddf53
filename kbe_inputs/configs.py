"""The five workloads: sizes and generator recipes (all synthetic and seeded).

C1 plain/small, C2 the headline norb=4 N_t=8192 case, C3 the batched lattice,
C4 reduced precision, C5 adjoint.  Only sizes and seeds live here.
"""
from __future__ import annotations

from .generators import hermitian_terms, lattice_terms, scalar_terms

CONFIGS = {
    "c1": dict(name="plain-small", norb=1, nt=512, h=0.02, k=5, leaf=32, tol=1e-10,
               nterms=8, seed_g=1, seed_s=2, beta_f=1.0),
    "c2": dict(name="norb4-nt8192", norb=4, nt=8192, h=0.01, k=5, leaf=64, tol=1e-10,
               nterms=8, seed_g=3, seed_s=4, beta_f=1.0),
    "c3": dict(name="lattice-32x32", norb=1, nt=2048, h=0.02, k=5, leaf=64, tol=1e-10,
               nk_side=32, seed=5, beta_f=1.0),
    "c4": dict(name="norb16-fp32proj", norb=16, nt=8192, h=0.01, k=5, leaf=64, tol=1e-6,
               nterms=12, seed_g=6, seed_s=7, beta_f=1.0),
    "c5": dict(name="adjoint-norb2", norb=2, nt=2048, h=0.02, k=5, leaf=64, tol=1e-10,
               nterms=8, seed_g=8, seed_s=9, beta_f=1.0, seed_w=10, ckpt=256),
}


def make_config_inputs(key: str, **override):
    """Return (cfg, G_params, Sigma_params) for a config; lists of per-k params for c3."""
    cfg = dict(CONFIGS[key])
    cfg.update(override)
    if key == "c3":
        g, s = lattice_terms(cfg["seed"], cfg["nk_side"], cfg["beta_f"])
        return cfg, g, s
    if cfg["norb"] == 1:
        g = scalar_terms(cfg["seed_g"], cfg["nterms"], cfg["beta_f"])
        s = scalar_terms(cfg["seed_s"], cfg["nterms"], cfg["beta_f"])
    else:
        g = hermitian_terms(cfg["seed_g"], cfg["nterms"], cfg["norb"], cfg["beta_f"])
        s = hermitian_terms(cfg["seed_s"], cfg["nterms"], cfg["norb"], cfg["beta_f"])
    return cfg, g, s
