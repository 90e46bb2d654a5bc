"""Pins for the oracle's AES-128 and CTR mode: FIPS-197 / SP 800-38A published
values (tests/golden) and the openssl command-line tool as an independent
implementation."""
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from conftest import golden


def test_fips197_block_vectors():
    for row in golden("fips197_aes128.txt"):
        if row[0] == "block":
            key, pt, ct = (bytes.fromhex(h) for h in row[1:])
            assert oracle.aes128_encrypt(key, pt) == ct


def test_fips197_key_schedule_words():
    for row in golden("fips197_aes128.txt"):
        if row[0] == "schedule":
            rk = oracle.aes_expand(bytes.fromhex(row[1]))
            i = int(row[2])
            assert rk[4 * i:4 * i + 4].hex() == row[3]


def test_sbox_entries_and_bijection():
    s = oracle.aes_sbox()
    for row in golden("fips197_aes128.txt"):
        if row[0] == "sbox":
            assert s[int(row[1], 16)] == int(row[2], 16)
    assert sorted(s.tolist()) == list(range(256))


def test_sp800_38a_ctr_vectors():
    rows = golden("sp800_38a_ctr_aes128.txt")
    key = bytes.fromhex([r for r in rows if r[0] == "key"][0][1])
    ctr0 = bytes.fromhex([r for r in rows if r[0] == "ctr0"][0][1])
    blocks = [r for r in rows if r[0] == "block"]
    pt = b"".join(bytes.fromhex(r[1]) for r in blocks)
    ct = b"".join(bytes.fromhex(r[2]) for r in blocks)
    assert oracle.ctr_xor(key, ctr0, pt).tobytes() == ct
    # starting at a block offset gives the matching suffix
    assert oracle.ctr_xor(key, ctr0, pt[32:], first_block=2).tobytes() == ct[32:]
    # truncated final block
    assert oracle.ctr_xor(key, ctr0, pt[:37]).tobytes() == ct[:37]


def _openssl(args, data):
    return subprocess.run(["openssl", "enc"] + args, input=data, capture_output=True, check=True).stdout


@pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl CLI not available")
def test_ctr_matches_openssl_random_and_carry():
    rng = np.random.default_rng(7)
    key = rng.integers(0, 256, 16, dtype=np.uint8).tobytes()
    data = rng.integers(0, 256, 16 * 300 + 5, dtype=np.uint8).tobytes()
    for ctr0 in (rng.integers(0, 256, 16, dtype=np.uint8).tobytes(),
                 bytes(7) + b"\x01" + b"\xff" * 8,       # carry out of the low 64 bits
                 b"\xff" * 16):                           # wrap-around mod 2^128
        ref = _openssl(["-aes-128-ctr", "-K", key.hex(), "-iv", ctr0.hex()], data)
        assert oracle.ctr_xor(key, ctr0, data).tobytes() == ref


@pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl CLI not available")
def test_ecb_matches_openssl():
    rng = np.random.default_rng(8)
    for _ in range(8):
        key = rng.integers(0, 256, 16, dtype=np.uint8).tobytes()
        blk = rng.integers(0, 256, 16, dtype=np.uint8).tobytes()
        assert oracle.aes128_encrypt(key, blk) == _openssl(["-aes-128-ecb", "-K", key.hex(), "-nopad"], blk)


def test_ctr_is_an_involution_and_errors_stay_local():
    # Sec. 6.10.8 of the report: a bit error in a protected part stays local.
    rng = np.random.default_rng(9)
    key = rng.integers(0, 256, 16, dtype=np.uint8).tobytes()
    ctr0 = rng.integers(0, 256, 16, dtype=np.uint8).tobytes()
    pt = rng.integers(0, 256, 1000, dtype=np.uint8)
    ct = oracle.ctr_xor(key, ctr0, pt)
    assert np.array_equal(oracle.ctr_xor(key, ctr0, ct), pt)
    bad = ct.copy()
    bad[123] ^= 0x10
    diff = oracle.ctr_xor(key, ctr0, bad) ^ pt
    assert np.count_nonzero(diff) == 1 and diff[123] == 0x10


def test_ctr_keystream_blocks_match_published_vector():
    rows = golden("sp800_38a_ctr_aes128.txt")
    key = bytes.fromhex([r for r in rows if r[0] == "key"][0][1])
    ctr0 = bytes.fromhex([r for r in rows if r[0] == "ctr0"][0][1])
    blocks = [r for r in rows if r[0] == "block"]
    ks = oracle.ctr_keystream(key, ctr0, [3, 0, 2, 1])
    for row, i in zip(ks, [3, 0, 2, 1]):
        pt, ct = bytes.fromhex(blocks[i][1]), bytes.fromhex(blocks[i][2])
        assert bytes(a ^ b for a, b in zip(row.tobytes(), pt)) == ct
