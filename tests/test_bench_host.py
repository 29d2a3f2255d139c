"""Host-side helpers of bench.py (no GPU): the kernel-source fingerprint that
ties committed counter figures to one version of the code, and the default
chunk layout the counter summary's algorithmic bytes are derived from."""
import os
import shutil

import bench


def test_source_hash_ignores_comments_but_not_code(tmp_path, monkeypatch):
    src = os.path.join(bench.ROOT, "paper_2011_03484_amd", "csrc")
    dst = tmp_path / "paper_2011_03484_amd" / "csrc"
    shutil.copytree(src, dst, ignore=shutil.ignore_patterns("__pycache__"))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    p = dst / "dmath.hpp"
    text = p.read_text()
    assert "return __builtin_fma(a, b, c);" in text
    p.write_text(text.replace("namespace tpm {", "namespace tpm {  // a note\n/* a block\n comment */\n", 1))
    assert bench.kernel_source_hash() == h0
    p.write_text(p.read_text().replace("return __builtin_fma(a, b, c);", "return __builtin_fma(b, a, c);"))
    assert bench.kernel_source_hash() != h0


def test_default_chunk_layout():
    assert bench.default_chunks(0) == []
    assert bench.default_chunks(500) == [500]
    assert bench.default_chunks(20000) == [1024, 8192, 8192, 2592]
    chunks = bench.default_chunks(1_000_000)
    assert sum(chunks) == 1_000_000 and len(chunks) == 123 and chunks[0] == 1024


def test_algorithmic_flops_match_the_oracle_tally(orc):
    """The roofline's algorithmic flops per particle-step are the oracle's own
    step tallied and weighted (oracle.count_ops / flops_per_step)."""
    from paper_2011_03484_amd import workloads as W
    w = W.giants_100k(n=200, seed=8)
    eph = orc.ephemeris(w.mu0, w.mu, w.rp, w.vp, 2, w.dt)
    c = orc.count_ops(w.mu0, w.mu, w.rcrit, w.rmax, eph.table, w.dt, w.r, w.v,
                      kepler_iters=w.kepler_iters)
    assert bench.ALGORITHMIC_FLOPS_PER_PARTICLE_STEP[w.np_] == orc.flops_per_step(c)
