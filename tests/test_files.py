"""Instance files with sha256 manifests and probing-cache files: round trips
and detection of altered contents (host only)."""
import json

import numpy as np
import pytest
import torch

from paper_2510_20499_amd import bp, gen


def test_instance_file_round_trip_and_manifest(tmp_path):
    inst = gen.make("tiny", 4)
    path = str(tmp_path / "tiny4.npz")
    d = gen.save(inst, path)
    assert d == gen.digest(inst)
    back = gen.load(path)
    assert gen.digest(back) == d
    for k in gen.ARRAYS + ("xstar",):
        assert np.array_equal(back[k], inst[k]) and back[k].dtype == np.asarray(inst[k]).dtype, k
    assert back["m"] == inst["m"] and back["n"] == inst["n"]
    man = json.load(open(path + ".sha256.json"))
    assert man["sha256"] == d and man["arrays"]["val"]["shape"] == [int(inst["row_ptr"][-1])]


def test_instance_file_detects_changes(tmp_path):
    inst = gen.make("tiny", 5)
    path = str(tmp_path / "tiny5.npz")
    gen.save(inst, path)
    other = dict(inst)
    other["val"] = inst["val"].copy()
    other["val"][3] += 1.0
    # the arrays written, the manifest of the original
    man = open(path + ".sha256.json").read()
    gen.save(other, path)
    open(path + ".sha256.json", "w").write(man)
    with pytest.raises(ValueError, match="val"):
        gen.load(path)
    assert gen.load(path, verify=False)["val"][3] == other["val"][3]
    bare = str(tmp_path / "bare.npz")
    open(bare, "wb").write(open(path, "rb").read())
    with pytest.raises(ValueError, match="no manifest"):
        gen.load(bare)


def test_digest_depends_on_every_array():
    inst = gen.make("tiny", 6)
    d = gen.digest(inst)
    for k in gen.ARRAYS:
        other = dict(inst)
        a = np.array(inst[k], copy=True)
        a.reshape(-1).view(np.uint8)[-1] ^= 1  # one bit of the last element
        other[k] = a
        assert gen.digest(other) != d, k


def _cache(k=3):
    rng = np.random.default_rng(1)
    cnt = rng.integers(0, 4, size=2 * k)
    off = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    tot = int(off[-1])
    return torch.arange(k, dtype=torch.int32) * 7, {
        "status": torch.tensor(rng.integers(0, 2, size=2 * k), dtype=torch.int8),
        "rounds": torch.tensor(rng.integers(0, 9, size=2 * k), dtype=torch.int32),
        "nnz": torch.tensor(rng.integers(0, 99, size=2 * k), dtype=torch.int64),
        "off": torch.from_numpy(off),
        "var": torch.tensor(rng.integers(0, 50, size=tot), dtype=torch.int32),
        "lb": torch.from_numpy(rng.uniform(0, 1, size=tot)),
        "ub": torch.from_numpy(rng.uniform(1, 2, size=tot)),
    }


def test_probe_cache_round_trip(tmp_path):
    vars_, out = _cache()
    path = str(tmp_path / "cache.npz")
    d = bp.save_probe_cache(path, vars_, out, instance_sha256="abc")
    back = bp.load_probe_cache(path, device="cpu", instance_sha256="abc")
    assert torch.equal(back["vars"], vars_)
    for k, t in out.items():
        assert torch.equal(back[k], t) and back[k].dtype == t.dtype, k
    assert json.load(open(path + ".sha256.json"))["sha256"] == d


def test_probe_cache_detects_changes_and_other_instances(tmp_path):
    vars_, out = _cache()
    path = str(tmp_path / "cache.npz")
    bp.save_probe_cache(path, vars_, out, instance_sha256="abc")
    with pytest.raises(ValueError, match="another instance"):
        bp.load_probe_cache(path, device="cpu", instance_sha256="def")
    man = open(path + ".sha256.json").read()
    out2 = dict(out)
    out2["lb"] = out["lb"].clone()
    out2["lb"][0] += 1e-12
    bp.save_probe_cache(path, vars_, out2, instance_sha256="abc")
    open(path + ".sha256.json", "w").write(man)
    with pytest.raises(ValueError, match="manifest"):
        bp.load_probe_cache(path, device="cpu")
