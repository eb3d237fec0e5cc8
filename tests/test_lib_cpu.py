"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, its host key function matches the oracle's Hilbert keys, its
FNV-1a matches the published definition, and argument errors are reported
without touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2607_20704_amd import _lib as L
from paper_2607_20704_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "rg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rg_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    syms = header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s
        assert s in L.SIGNATURES, "binding lacks " + s


def test_abi_version_and_status_strings():
    lib = L.lib()
    with open(os.path.join(ROOT, "include", "rg.h")) as f:
        declared = int(re.search(r"#define RG_ABI_VERSION (\d+)", f.read()).group(1))
    assert lib.rg_abi_version() == declared
    assert lib.rg_status_string(L.RG_EUNGRADED) == b"RG_EUNGRADED"
    assert lib.rg_status_string(99) == b"RG_UNKNOWN"


def fnv1a64_bytes(data):
    """FNV-1a 64 from the published definition: offset basis, then for each
    byte xor and multiply by the FNV prime modulo 2^64."""
    h = 0xCBF29CE484222325
    for b in data:
        h ^= b
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def test_fnv_reference_vectors():
    # published FNV-1a 64 test vectors
    assert fnv1a64_bytes(b"") == 0xCBF29CE484222325
    assert fnv1a64_bytes(b"a") == 0xAF63DC4C8601EC8C
    assert fnv1a64_bytes(b"foobar") == 0x85944171F73967E8


def test_library_fnv_hashes_the_8_key_bytes():
    rng = np.random.default_rng(4)
    for K in [1, 8, 0x1234, 2 ** 60 + 12345] + [int(x) for x in rng.integers(1, 2 ** 62, 50)]:
        assert api.fnv1a64(K) == fnv1a64_bytes(int(K).to_bytes(8, "little"))


@pytest.mark.parametrize("l", [1, 2, 3, 4, 5, 6])
def test_host_keys_equal_oracle_keys_exhaustive(l):
    n = 1 << (l - 1)
    for i in range(n):
        for j in range(n):
            for k in range(0, n, max(1, n // 8)):
                K = api.key_host(i, j, k, l)
                assert K == O.key(i, j, k, l)
                assert api.key_coords_host(K) == (i, j, k, l)


def test_host_keys_equal_oracle_keys_deep():
    rng = np.random.default_rng(5)
    for l in range(7, 22):
        n = 1 << (l - 1)
        for _ in range(100):
            i, j, k = (int(x) for x in rng.integers(0, n, 3))
            K = api.key_host(i, j, k, l)
            assert K == O.key(i, j, k, l)
            assert api.key_coords_host(K) == (i, j, k, l)


def test_out_of_range_coordinates_give_key_zero():
    assert api.key_host(4, 0, 0, 3) == 0
    assert api.key_host(0, -1, 0, 3) == 0
    assert api.key_host(0, 0, 0, 0) == 0
    assert api.key_host(0, 0, 0, 22) == 0


def test_argument_errors_are_reported_without_a_device():
    lib = L.lib()
    assert lib.rg_encode_keys(None, 5, None, None) == L.RG_EINVAL
    assert b"null pointer" in L.detail().encode()
    assert lib.rg_hash_build(None, -1, None, 0, None) == L.RG_EINVAL
    # a workspace that is too small is refused before anything is enqueued
    fake = ctypes.c_void_p(256)
    assert lib.rg_hash_build(fake, 100, fake, 64, None) == L.RG_EFULL
    assert lib.rg_build_neighbours(fake, fake, 10, 1, 7, fake, fake, fake, None) == L.RG_EINVAL
    assert lib.rg_hydro_step_level(1.0, None, 1.4, None, None, None, None, 0, 10, None, 0, 0.8, None, 0, None,
                                   None) == L.RG_EINVAL
    assert lib.rg_hydro_step_level(1.0, fake, 1.4, fake, fake, fake, fake, 0, 10, None, 0, 0.8, None, 5, None,
                                   None) == L.RG_EINVAL
    # a fused time step needs a positive CFL number
    assert lib.rg_hydro_step_level(1.0, fake, 1.4, fake, ctypes.c_void_p(512), fake, fake, 0, 10, None, 0, 0.0,
                                   fake, 0, None, None) == L.RG_EINVAL
    assert lib.rg_cfl_dt_corrected(None, None, None, 1, 2, 1.4, 0.8, None, None) == L.RG_EINVAL
    lb = (ctypes.c_int64 * 23)()
    assert lib.rg_cfl_dt(fake, fake, lb, 3, 2, 1.4, 0.8, fake, None) == L.RG_EINVAL
    assert lib.rg_step(None, None, None, 1.4, 0.8, 0, 0, None, None, None) == L.RG_EINVAL
    # zero-sized work is a no-op
    assert lib.rg_encode_keys(None, 0, None, None) == L.RG_OK


def test_batch_argument_errors_without_a_device():
    """rg_batch_create validates every tree on the host before any device
    call; rg_batch_run refuses a null batch and rg_batch_destroy accepts one."""
    lib = L.lib()
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(256)
    assert lib.rg_batch_create(None, 1, 0, 2, 0, None, fake, None, ctypes.byref(out)) == L.RG_EINVAL
    tree = L.RgTree()
    tree.n_oct, tree.lmin, tree.lmax = 8, 2, 2
    bt = (L.RgBatchTree * 1)()
    bt[0].tree = ctypes.pointer(tree)
    bt[0].d_u0, bt[0].d_u1, bt[0].gamma, bt[0].cfl = 256, 512, 1.4, 0.8
    # no schedule
    assert lib.rg_batch_create(bt, 1, 0, 2, 0, None, fake, None, ctypes.byref(out)) == L.RG_EINVAL
    assert b"schedule" in L.detail().encode()
    sched = L.RgSchedule()
    sched.d_list = 1024
    tree.sched = ctypes.pointer(sched)
    # bad form, flags, step count, group size, aliasing state buffers
    assert lib.rg_batch_create(bt, 1, 7, 2, 0, None, fake, None, ctypes.byref(out)) == L.RG_EINVAL
    assert lib.rg_batch_create(bt, 1, 0, 2, L.RG_STEP_REKEY, None, fake, None, ctypes.byref(out)) == L.RG_EINVAL
    assert lib.rg_batch_create(bt, 1, 0, 0, 0, None, fake, None, ctypes.byref(out)) == L.RG_EINVAL
    tune = L.RgTuning()
    tune.octs_per_group = 3
    assert lib.rg_batch_create(bt, 1, 0, 2, 0, ctypes.byref(tune), fake, None, ctypes.byref(out)) == L.RG_EINVAL
    bt[0].d_u1 = 256
    assert lib.rg_batch_create(bt, 1, 0, 2, 0, None, fake, None, ctypes.byref(out)) == L.RG_EINVAL
    assert out.value is None
    assert lib.rg_batch_run(None, None) == L.RG_EINVAL
    assert lib.rg_batch_destroy(None) == L.RG_OK


def test_subcycled_step_argument_errors_without_a_device():
    """rg_step_subcycled checks its arguments on the host first."""
    lib = L.lib()
    tree = L.RgTree()
    tree.n_oct, tree.lmin, tree.lmax = 72, 2, 3
    tree.level_begin[2], tree.level_begin[3], tree.level_begin[4] = 0, 8, 72
    u, scratch, acc, dt = 256, 512, 768, 1024
    ok = (ctypes.byref(tree), u, scratch, acc, 1.4, 0.8, 0, 0, dt, None, None)

    def call(**kw):
        a = list(ok)
        for k, v in kw.items():
            a[["t", "u", "scratch", "acc", "gamma", "cfl", "form", "flags", "dt", "tune", "stream"].index(k)] = v
        return lib.rg_step_subcycled(*a)

    assert call(t=None) == L.RG_EINVAL
    assert call(dt=None) == L.RG_EINVAL
    # a multilevel tree needs the accumulation buffer
    assert call(acc=None) == L.RG_EINVAL
    assert b"accumulation" in L.detail().encode()
    assert call(scratch=u) == L.RG_EINVAL
    assert b"alias" in L.detail().encode()
    assert call(flags=L.RG_STEP_CHAIN_DT) == L.RG_EINVAL
    assert call(form=9) == L.RG_EINVAL
    assert call(gamma=1.0) == L.RG_EINVAL
    assert call(cfl=0.0) == L.RG_EINVAL
    assert call(u=257) == L.RG_EINVAL
    tree.level_begin[4] = 71
    assert call() == L.RG_EINVAL


def test_refine_argument_errors_without_a_device():
    """rg_refine and rg_refine_flags check the tree, the parameters, the
    buffers and the capacity on the host before any device call."""
    lib = L.lib()
    tree = L.RgTree()
    tree.n_oct, tree.lmin, tree.lmax = 72, 2, 3
    tree.level_begin[2], tree.level_begin[3], tree.level_begin[4] = 0, 8, 72
    tree.d_nbr27, tree.d_father_cell, tree.d_son_mask = 256, 512, 768
    p = L.RgRefineParams()
    p.rho_thresh, p.grad_thresh, p.lmax = 1.0, 0.0, 5
    u, u2, ws = 1024, 2048, 4096
    assert lib.rg_refine_flags(None, u, ctypes.byref(p), 1, ws, None) == L.RG_EINVAL
    assert lib.rg_refine_flags(ctypes.byref(tree), None, ctypes.byref(p), 1, ws, None) == L.RG_EINVAL
    p.lmax = 1
    assert lib.rg_refine_flags(ctypes.byref(tree), u, ctypes.byref(p), 1, ws, None) == L.RG_EINVAL
    p.lmax = 5
    p.nsubgrid = 3
    assert lib.rg_refine_flags(ctypes.byref(tree), u, ctypes.byref(p), 1, ws, None) == L.RG_EINVAL
    p.nsubgrid = 4
    need = lib.rg_refine_workspace_bytes(72)
    assert need > 72 * 4 * 5
    assert lib.rg_refine(ctypes.byref(tree), u, u, ctypes.byref(p), ws, need, None) == L.RG_EINVAL
    # no coordinates / scratch / sort workspace
    assert lib.rg_refine(ctypes.byref(tree), u, u2, ctypes.byref(p), ws, need, None) == L.RG_EINVAL
    tree.d_ijkl, tree.d_keys_scratch, tree.d_perm, tree.d_sort_ws = 8192, 16384, 32768, 65536
    tree.d_level_begin, tree.d_hash_ws = 131072, 262144
    tree.sort_ws_bytes = lib.rg_sort_workspace_bytes(72)
    tree.hash_ws_bytes = lib.rg_hash_workspace_bytes(72)
    tree.capacity = 64       # below n_oct
    assert lib.rg_refine(ctypes.byref(tree), u, u2, ctypes.byref(p), ws, need, None) == L.RG_EINVAL
    assert b"capacity" in L.detail().encode()
    tree.capacity = 200      # workspaces sized for 72 octs only
    assert lib.rg_refine(ctypes.byref(tree), u, u2, ctypes.byref(p), ws, need, None) == L.RG_EINVAL
    tree.capacity = 0
    assert lib.rg_refine(ctypes.byref(tree), u, u2, ctypes.byref(p), ws, need - 256, None) == L.RG_EINVAL
    assert lib.rg_refine(ctypes.byref(tree), u, u2, ctypes.byref(p), ws + 8, need, None) == L.RG_EINVAL


def test_multigrid_argument_errors_without_a_device():
    """rg_mg_vcycles checks the hierarchy on the host: periodic, levels
    present and complete, sane counts."""
    lib = L.lib()
    tree = L.RgTree()
    tree.n_oct, tree.lmin, tree.lmax, tree.bc = 73, 1, 3, 0
    for l, b in ((1, 0), (2, 1), (3, 9), (4, 73)):
        tree.level_begin[l] = b
    tree.d_nbr27, tree.d_father_cell = 256, 512
    a = (256, 512, 768)
    assert lib.rg_mg_vcycles(ctypes.byref(tree), *a, 3, 1, 2, 2, 10, 0, None) == L.RG_OK   # zero cycles
    assert lib.rg_mg_vcycles(ctypes.byref(tree), *a, 4, 1, 2, 2, 10, 1, None) == L.RG_EINVAL
    assert lib.rg_mg_vcycles(ctypes.byref(tree), *a, 3, 0, 2, 2, 10, 1, None) == L.RG_EINVAL
    assert lib.rg_mg_vcycles(ctypes.byref(tree), *a, 3, 1, -1, 2, 10, 1, None) == L.RG_EINVAL
    assert lib.rg_mg_vcycles(ctypes.byref(tree), None, 512, 768, 3, 1, 2, 2, 10, 1, None) == L.RG_EINVAL
    tree.level_begin[3] = 8      # level 2 incomplete
    assert lib.rg_mg_vcycles(ctypes.byref(tree), *a, 3, 1, 2, 2, 10, 1, None) == L.RG_EINVAL
    tree.level_begin[3] = 9
    tree.bc = 1
    assert lib.rg_mg_vcycles(ctypes.byref(tree), *a, 3, 1, 2, 2, 10, 1, None) == L.RG_EINVAL
    assert b"periodic" in L.detail().encode()


def test_workspace_sizes():
    lib = L.lib()
    # the table (256-byte header, capacity = power of two >= 2n slots of 12
    # bytes) followed by the scratch of the segmented build (the bucketed
    # keys, two int32 arrays of n entries, the per-chunk segment counts, the
    # segment bounds)
    def table(cap):
        return (256 + cap * 12 + 255) // 256 * 256
    for n, cap in ((0, 16), (4096, 8192), (4097, 16384), (1 << 21, 1 << 22)):
        b = lib.rg_hash_workspace_bytes(n)
        assert b >= table(cap) + 16 * n, (n, b)
        assert b % 256 == 0
        assert b < table(cap) + 16 * n + 2 * n + 64 * 1024, (n, b)
    assert lib.rg_corr_workspace_bytes(10) == 2400
