"""Tile steps specialised at run time (each step compiled into a kernel of
its own by the ROCm clang): the same results as the generic tile kernel, bit
for bit, and parity with the FP64 oracle; the on-disk code-object cache."""
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, amp_err, banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs():
    import paper_2311_01512_amd as pkg
    return pkg


@pytest.mark.parametrize("prec,k", [("c64", 12), ("c128", 11), ("c64", 10), ("c128", 12), ("c128", 13)])
def test_specialized_equals_generic_and_oracle(qs, prec, k):
    banner(f"specialised tiles {prec} k={k}")
    N = 14
    ops = synth.config2_circuit(num_qubits=N, num_gates=160)
    rng = np.random.default_rng(71)
    psi = synth.random_state(rng, 1 << N)
    c = qs.Circuit(N, ops).compile(k, prec)
    q = qs.Qureg(N, precision=prec).set_amps(psi)
    c.apply(q)
    generic = q.get_amps()
    nk = c.specialize()
    assert nk > 0
    q.set_amps(psi)
    c.apply(q)
    special = q.get_amps()
    assert np.array_equal(special, generic)
    assert amp_err(special, oracle.run_ops(psi.copy(), ops)) < TOL[prec]


@pytest.mark.parametrize("N,k,prec,seed", [(24, 12, "c64", 11), (22, 10, "c64", 5), (20, 13, "c64", 11),
                                           (24, 11, "c128", 11), (23, 12, "c128", 7), (22, 13, "c128", 11)])
def test_every_specialized_pass_equals_generic(qs, N, k, prec, seed):
    """Each step of a 500-gate circuit on a state with many tiles, applied by
    its own kernel and by the generic one to the same input, bit for bit.
    (Steps with controls on tile-base qubits once came out wrong when the
    prefetch registers were left undefined after the last tile.)"""
    banner(f"every specialised pass N={N} k={k} {prec} seed={seed}")
    import torch
    ops = synth.config2_circuit(num_qubits=N, num_gates=500, seed=seed)
    cg = qs.Circuit(N, ops).compile(k, prec)
    cs = qs.Circuit(N, ops).compile(k, prec)
    assert cs.specialize() > 0
    qg = qs.Qureg(N, precision=prec).init_hashed(7)
    qx = qs.Qureg(N, precision=prec)
    bad = []
    for i in range(cg.stats()["num_passes"]):
        qx.tensor.copy_(qg.tensor)
        cg.apply_passes(qg, i, 1)
        cs.apply_passes(qx, i, 1)
        qx.sync()
        qg.sync()
        if not torch.equal(qg.tensor, qx.tensor):
            bad.append(i)
    assert bad == []


@pytest.mark.parametrize("k", [11, 12])
def test_every_specialized_density_pass_equals_generic(qs, k):
    """Density steps with matrix-core superoperators, whose coefficients the
    specialised kernels stage in LDS: each step bit for bit against the
    generic kernel on an 11-qubit density matrix (22 index bits)."""
    banner(f"every specialised density pass k={k}")
    import torch
    N = 11
    ops, _ = synth.config3_circuit(num_qubits=N, num_ops=200, seed=76)
    cg = qs.Circuit(N, ops, density=True).compile(k, "c64")
    cs = qs.Circuit(N, ops, density=True).compile(k, "c64")
    assert cs.specialize() > 0
    qg = qs.Qureg(N, density=True, precision="c64").init_hashed(7)
    qx = qs.Qureg(N, density=True, precision="c64")
    bad = []
    for i in range(cg.stats()["num_passes"]):
        qx.tensor.copy_(qg.tensor)
        cg.apply_passes(qg, i, 1)
        cs.apply_passes(qx, i, 1)
        qx.sync()
        qg.sync()
        if not torch.equal(qg.tensor, qx.tensor):
            bad.append(i)
    assert bad == []


def test_specialized_density_circuit(qs):
    """A density circuit with Kraus maps as sparse and matrix-core operators."""
    banner("specialised density circuit")
    N = 7
    ops, _ = synth.config3_circuit(num_qubits=N, num_ops=80)
    rng = np.random.default_rng(72)
    psi = synth.random_state(rng, 1 << N)
    rho = np.outer(psi, psi.conj()).reshape(-1, order="F")
    c = qs.Circuit(N, ops, density=True).compile(12, "c64")
    q = qs.Qureg(N, density=True, precision="c64").set_amps(rho)
    c.apply(q)
    generic = q.get_amps()
    c.specialize()
    q.set_amps(rho)
    c.apply(q)
    assert np.array_equal(q.get_amps(), generic)
    assert amp_err(q.get_amps(), oracle.run_ops(rho.copy(), ops, density=True)) < TOL["c64"]


def test_recompile_drops_specialization(qs):
    banner("recompile after specialise")
    N = 12
    ops = synth.config2_circuit(num_qubits=N, num_gates=60)
    rng = np.random.default_rng(73)
    psi = synth.random_state(rng, 1 << N)
    c = qs.Circuit(N, ops).compile(11, "c64")
    c.specialize()
    c.compile(10, "c64")            # new passes: the specialised kernels are gone
    q = qs.Qureg(N, precision="c64").set_amps(psi)
    c.apply(q)
    assert amp_err(q.get_amps(), oracle.run_ops(psi.copy(), ops)) < TOL["c64"]
    assert qs.Circuit(N, ops).compile(0, "c64").specialize() == 0   # no tile steps


def test_disk_cache(qs, tmp_path, monkeypatch):
    """Code objects land in $QS_JIT_CACHE as files that start with their
    whole compilation key; a second circuit with the same steps loads them."""
    banner("specialised tiles: disk cache")
    monkeypatch.setenv("QS_JIT_CACHE", str(tmp_path))
    N = 13
    ops = synth.config2_circuit(num_qubits=N, num_gates=70, seed=74)
    rng = np.random.default_rng(74)
    psi = synth.random_state(rng, 1 << N)
    c = qs.Circuit(N, ops).compile(12, "c64")
    q = qs.Qureg(N, precision="c64").set_amps(psi)
    c.apply(q)
    generic = q.get_amps()
    assert c.specialize() > 0
    files = sorted(os.listdir(tmp_path))
    assert files and all(f.endswith(".co") for f in files)
    for f in files:
        blob = (tmp_path / f).read_bytes()
        assert b"qs_step_" in blob.split(b"\0", 1)[0]      # the key holds the generated source
    c2 = qs.Circuit(N, ops).compile(12, "c64")
    assert c2.specialize() > 0
    assert sorted(os.listdir(tmp_path)) == files
    q.set_amps(psi)
    c2.apply(q)
    assert np.array_equal(q.get_amps(), generic)


def test_whole_circuit_equals_generic(qs):
    """Two applications of a 24-qubit circuit: the specialised steps round
    exactly as the generic kernel does (no implicit contraction of products
    into sums in either build)."""
    banner("whole circuit, specialised vs generic")
    import torch
    N = 24
    ops = synth.config2_circuit(num_qubits=N, num_gates=500)
    cg = qs.Circuit(N, ops).compile(12, "c64")
    cs = qs.Circuit(N, ops).compile(12, "c64")
    cs.specialize()
    qg = qs.Qureg(N, precision="c64").init_hashed(7)
    qx = qs.Qureg(N, precision="c64").init_hashed(7)
    for _ in range(2):
        cg.apply(qg)
        cs.apply(qx)
    qg.sync()
    qx.sync()
    assert torch.equal(qg.tensor, qx.tensor)


def test_autotune_with_specialised_steps(qs):
    """The autotuner times tile widths generic and specialised and leaves the
    circuit in the fastest form; the result still matches the oracle."""
    banner("autotune with specialised steps")
    N = 14
    ops = synth.config2_circuit(num_qubits=N, num_gates=120, seed=75)
    rng = np.random.default_rng(75)
    psi = synth.random_state(rng, 1 << N)
    c = qs.Circuit(N, ops)
    q = qs.Qureg(N, precision="c64").init_zero()
    best, ms, ms_spec = c.autotune(q, (0, 4, 11, 12), specialize=True)
    assert best in (0, 4, 11, 12)
    assert set(ms) == {0, 4, 11, 12}
    assert set(ms_spec) == {11, 12}                  # only tile widths have a specialised form
    assert all(v > 0 for v in ms_spec.values())
    fastest = min(min(ms.values()), min(ms_spec.values()))
    chosen = ms_spec[best] if c.specialized else ms[best]
    assert chosen == fastest
    q.set_amps(psi)
    c.apply(q)
    assert amp_err(q.get_amps(), oracle.run_ops(psi.copy(), ops)) < TOL["c64"]
    best2, _ = c.autotune(q, (0, 4))                 # the plain autotuner: no specialised steps
    assert c.specialized == 0 and best2 in (0, 4)


@pytest.mark.parametrize("N,k,prec", [(9, 13, "c64"), (10, 10, "c64"), (12, 13, "c128"), (13, 13, "c64")])
def test_specialized_single_tile_and_clipped_width(qs, N, k, prec):
    """Tile width at or above the qubit count: one tile holds the whole state
    (a single block walks it), the width is clipped to N."""
    banner(f"specialised one-tile N={N} k={k} {prec}")
    ops = synth.config2_circuit(num_qubits=N, num_gates=90, seed=77 + N)
    rng = np.random.default_rng(77 + N)
    psi = synth.random_state(rng, 1 << N)
    c = qs.Circuit(N, ops).compile(k, prec)
    q = qs.Qureg(N, precision=prec).set_amps(psi)
    c.apply(q)
    generic = q.get_amps()
    assert c.specialize() > 0
    q.set_amps(psi)
    c.apply(q)
    assert np.array_equal(q.get_amps(), generic)
    assert amp_err(q.get_amps(), oracle.run_ops(psi.copy(), ops)) < TOL[prec]


def test_specialized_density_circuit_c128(qs):
    """Complex128 density circuit: superoperators in registers and sparse form
    (no matrix cores in double precision)."""
    banner("specialised density circuit c128")
    N = 6
    ops, _ = synth.config3_circuit(num_qubits=N, num_ops=60, seed=78, num_traced=3)
    rng = np.random.default_rng(78)
    psi = synth.random_state(rng, 1 << N)
    rho = np.outer(psi, psi.conj()).reshape(-1, order="F")
    c = qs.Circuit(N, ops, density=True).compile(11, "c128")
    q = qs.Qureg(N, density=True, precision="c128").set_amps(rho)
    c.apply(q)
    generic = q.get_amps()
    assert c.specialize() > 0
    q.set_amps(rho)
    c.apply(q)
    assert np.array_equal(q.get_amps(), generic)
    assert amp_err(q.get_amps(), oracle.run_ops(rho.copy(), ops, density=True)) < TOL["c128"]


def test_circuit_dropped_while_its_steps_are_queued(qs):
    """A specialised circuit applied several times asynchronously and then
    destroyed at once: destruction waits for the queued steps before it
    frees their tables and unloads their kernels, so the result equals that
    of a circuit kept alive."""
    import torch
    banner("circuit dropped with queued steps")
    n = 22
    ops = synth.config2_circuit(num_qubits=n, num_gates=300, seed=7)
    ref = qs.Qureg(n, precision="c64").init_hashed(3)
    keep = qs.Circuit(n, ops).compile(12, "c64")
    assert keep.specialize() > 0
    for _ in range(3):
        keep.apply(ref)
    ref.sync()
    q = qs.Qureg(n, precision="c64").init_hashed(3)
    c = qs.Circuit(n, ops).compile(12, "c64")
    assert c.specialize() > 0
    for _ in range(3):
        c.apply(q)
    c.close()          # no sync before: the steps are still queued
    del c
    q.sync()
    assert torch.equal(q.tensor, ref.tensor)


def test_circuit_recompiled_while_its_steps_are_queued(qs):
    """Recompiling and re-specialising a circuit right after queueing its
    steps: the old tables and kernels stay until those steps have run."""
    import torch
    banner("circuit recompiled with queued steps")
    n = 21
    ops = synth.config2_circuit(num_qubits=n, num_gates=200, seed=8)
    ref = qs.Qureg(n, precision="c64").init_hashed(4)
    keep = qs.Circuit(n, ops).compile(12, "c64")
    keep.specialize()
    keep.apply(ref)
    keep.apply(ref)
    ref.sync()
    q = qs.Qureg(n, precision="c64").init_hashed(4)
    c = qs.Circuit(n, ops).compile(12, "c64")
    c.specialize()
    c.apply(q)
    c.compile(12, "c64")      # frees the tables the queued steps read
    c.specialize()
    c.apply(q)
    q.sync()
    assert torch.equal(q.tensor, ref.tensor)
