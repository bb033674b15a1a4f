"""Library and model files on the host (no GPU): files written here by the
format documented in include/hyperoms.h, with this test's own checksum code,
are read back by homs_file_inspect; a damaged, truncated or padded file and a
foreign file are refused."""
import os
import struct

import numpy as np
import pytest

from conftest import ROOT


@pytest.fixture(scope="module")
def h():
    lib = os.path.join(ROOT, "paper_2211_16422_amd", "libhyperoms.so")
    if not os.path.exists(lib):
        from paper_2211_16422_amd.build import build
        build()
    import paper_2211_16422_amd.hyperoms as mod
    return mod


def checksum(data: bytes) -> int:
    """FNV-1a over little-endian 64-bit words, the last one zero-padded."""
    h = 0xcbf29ce484222325
    pad = (-len(data)) % 8
    words = np.frombuffer(data + b"\0" * pad, dtype="<u8")
    for w in words.tolist():
        h = ((h ^ w) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def test_checksum_of_known_words():
    # one word: (offset ^ w) * prime; an empty input leaves the offset basis
    assert checksum(b"") == 0xcbf29ce484222325
    w = 0x0102030405060708
    assert checksum(struct.pack("<Q", w)) == ((0xcbf29ce484222325 ^ w) * 0x100000001b3) % 2 ** 64
    assert checksum(b"\x01") == checksum(struct.pack("<Q", 1))


def library_bytes(n, dim, seed=1, hash_=0x1234, charge_match=1):
    rng = np.random.default_rng(seed)
    head = b"HOMSLIB1" + struct.pack("<8I", 1, dim, 16, 50, dim // 2, charge_match, 0, 0)
    head += struct.pack("<4d", 101.0, 1500.0, 20.0, 0.01)
    head += struct.pack("<QQq", 7, hash_, n)
    assert len(head) == 96
    orig = rng.permutation(n).astype("<u4")
    pmz = np.sort(rng.uniform(400, 1500, n)).astype("<f8")
    charge = np.full(n, 2, np.int8)
    hv = rng.integers(0, 2 ** 32, (n, dim // 32), dtype=np.uint64).astype("<u4")
    body = head + orig.tobytes() + pmz.tobytes() + charge.tobytes() + hv.tobytes()
    return body + struct.pack("<Q", checksum(body))


def model_bytes(dim, hidden, embed, step=11, seed=2):
    rng = np.random.default_rng(seed)
    head = b"HOMSMDL1" + struct.pack("<2I2iq", 1, dim, hidden, embed, step)
    assert len(head) == 32
    sizes = [hidden * dim, hidden, embed * hidden, embed]
    arrays = [rng.normal(size=k).astype("<f4") for k in sizes * 3]
    body = head + b"".join(a.tobytes() for a in arrays)
    return body + struct.pack("<Q", checksum(body))


def test_library_file_is_read(h, tmp_path):
    p = tmp_path / "lib.homs"
    p.write_bytes(library_bytes(37, 1024, hash_=0xDEADBEEF12345678))
    info = h.file_info(str(p))
    assert info["kind"] == h.FILE_LIBRARY and info["version"] == 1
    assert info["dim"] == 1024 and info["n"] == 37
    assert info["codebook_hash"] == 0xDEADBEEF12345678
    prm = info["params"]
    assert (prm["n_levels"], prm["top_n"], prm["id_flips"], prm["seed"]) == (16, 50, 512, 7)
    assert prm["bins_per_da"] == 20.0 and prm["charge_match"] == 1


def test_model_file_is_read(h, tmp_path):
    p = tmp_path / "m.homs"
    p.write_bytes(model_bytes(512, 64, 32, step=11))
    info = h.file_info(str(p))
    assert info["kind"] == h.FILE_MODEL
    assert (info["dim"], info["hidden"], info["embed"], info["step"]) == (512, 64, 32, 11)


@pytest.mark.parametrize("damage", ["flip", "truncate", "extend", "magic", "size"])
def test_damaged_files_are_refused(h, tmp_path, damage):
    data = bytearray(library_bytes(20, 512))
    if damage == "flip":
        data[200] ^= 0x10
    elif damage == "truncate":
        data = data[:-3]
    elif damage == "extend":
        data += b"\0"
    elif damage == "magic":
        data[0:8] = b"NOTAHOMS"
    elif damage == "size":  # header claims one more row than the file holds
        data[88:96] = struct.pack("<q", 21)
    p = tmp_path / "bad.homs"
    p.write_bytes(bytes(data))
    with pytest.raises(h.HomsError) as e:
        h.file_info(str(p))
    assert e.value.status == h.HOMS_E_INVALID
    with pytest.raises(h.HomsError):
        h.file_info(str(tmp_path / "missing.homs"))
