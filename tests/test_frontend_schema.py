"""Host-side checks of the front end's gate schema (no GPU): every entry
names a library kind with matching arity, and the functional, module and
device-method forms are generated for every entry."""

import torch

from paper_2511_19291_amd import circuits as C
from paper_2511_19291_amd import frontend as F


def test_schema_matches_library_kinds():
    for name, (kind, nc, nt, npar) in F.GATE_SCHEMA.items():
        assert kind in C.ALL_KINDS, name
        assert C.N_TARGETS[kind] == nt and C.N_PARAMS[kind] == npar, name
        assert 0 <= nc <= 3


def test_forms_generated_for_every_entry():
    for name, (_, nc, nt, npar) in F.GATE_SCHEMA.items():
        assert callable(getattr(F.functional, name))
        cls = F.MODULES[name]
        assert cls.__name__ == name.upper() and getattr(F, name.upper()) is cls
        m = cls(wires=list(range(nc + nt)))
        if npar:
            assert isinstance(m.params, torch.nn.Parameter) and m.params.shape == (npar,)
            assert 0 <= float(m.params.detach().min()) and float(m.params.detach().max()) < 2 * 3.1416
        else:
            assert m.params is None
        frozen = cls(wires=list(range(nc + nt)), trainable=False, init_params=[0.5] * npar if npar else None)
        assert not any(p.requires_grad for p in frozen.parameters())


def test_ring_ansatz_structure_builds_on_cpu():
    nq, layers = 5, 4
    mod = F.ring_ansatz(nq, layers, rotation="rz")
    assert isinstance(mod.layers[0], F.GeneralEncoder)
    names = [m.name for m in mod.layers[1:]]
    assert names == (["rz"] * nq + ["cx"] * nq) * layers
    assert sum(p.numel() for p in mod.parameters()) == layers * nq
    rings = [m.wires for m in mod.layers[1:] if m.name == "cx"][:nq]
    assert rings == [[w, (w + 1) % nq] for w in range(nq)]
