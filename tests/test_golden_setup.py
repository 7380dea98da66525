"""The defaults and workloads against the set-up the paper states
(tests/golden/paper_setup.json, each value with its passage)."""
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def golden():
    return {k: v["value"] for k, v in
            json.load(open(os.path.join(HERE, "golden", "paper_setup.json")))["values"].items()}


def test_default_cutoffs_are_the_papers():
    from paper_1503_01722_amd import omc
    g = golden()
    p = omc.default_params()
    assert (p.Eabs_e, p.Eabs_g, p.kc, p.Wcc) == (g["Eabs_e_MeV"], g["Eabs_g_MeV"], g["kc_MeV"],
                                                 g["Wcc_MeV"])


def test_workloads_follow_the_papers_setup(W):
    g = golden()
    ph, src, _ = W.config("slab_6mv")
    assert ph["voxel"] == (g["voxel_cm"],) * 3
    assert all(n * h == g["phantom_side_cm"] for n, h in zip(ph["shape"], ph["voxel"]))
    assert src["ssd"] == g["ssd_cm"] and src["geometry"] == 1
    # the layers along z, from the surface: water, bone, lung, water
    names = [ph["materials"][m]["name"] for m in ph["material"][:, 0, 0]]
    layers = [names[0]] + [b for a, b in zip(names, names[1:]) if a != b]
    assert layers == g["slab_layers"]
    # the 6 MV spectrum ends at 6 MeV
    assert np.isclose(src["edges"][-1], float(g["photon_MV"]))
    _, e15, _ = W.config("halfslab_e15")
    assert e15["mono_E"] == g["electron_MeV"] and e15["ssd"] == g["ssd_cm"]
    assert len(W.MATERIALS_16) == g["n_materials"]
