"""CPU replay of the LDS index arithmetic of the column-MLP kernels
(mlp_infer_kernel, gemm_rows_kernel): between two workgroup barriers no
LDS byte written by one wave is read or written by another, and every
access stays inside its array.  The replay restates the kernels' index
expressions; the first test checks that the source still holds them, so a
change of the kernels' LDS layout fails here until the replay follows."""
import os

import numpy as np

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2504_08157_amd", "csrc", "nh_mlp.hip")
HDR = os.path.join(os.path.dirname(__file__), "..", "paper_2504_08157_amd", "csrc", "nh_internal.h")

IN, HID, NC = 208, 256, 65
NF = 3 * NC
LDF, LDH = IN + 8, HID + 8
REG = 64 * (NF + 1) * 4     # bytes of the shared region (features, H1, H2, outputs)
NWV = 8                     # waves of the inference workgroup


def test_source_holds_the_replayed_expressions():
    src = open(SRC).read()
    hdr = open(HDR).read()
    for s in ("constexpr int kMlpIn = 208;", "constexpr int kMlpHid = 256;", "constexpr int kMlpNC = 65;",
              "constexpr int kMlpNF = 3 * kMlpNC;"):
        assert s in hdr, s
    for s in ("constexpr int kLdF = kMlpIn + 8;", "constexpr int kLdH = kMlpHid + 8;",
              "constexpr int kRegBytes = 64 * (kMlpNF + 1) * 4;",
              "_Float16 *fr = sf + lane * kLdF;",
              "for (int c = q; c < kMlpNC; c += NWV) {",
              "fr[f * kMlpNC + c] = (_Float16)(vl / s);",
              "fr[kMlpNF + 2] = (_Float16)(log10(H) / 5.0);",
              "for (int i = kMlpNF + 3; i < kMlpIn; ++i) fr[i] = (_Float16)0.0f;",
              "av[a] = *(const half8 *)(S + (16 * a + r16) * ld + k + 8 * g);",
              "av[a] = *(const half4 *)(S + (16 * a + r16) * ld + K32 + 4 * g);",
              "const int row = 16 * a + 4 * g + i, cl = 32 * wave + 16 * c + r16;",
              "sh[row * kLdH + cl] = (_Float16)(z / (1.0f + expf(-z)));",
              "if (cl < kMlpNF) sy[row * (kMlpNF + 1) + cl] = acc3[a][c][i] + wt.bias[2][cl];",
              "const float *yr = sy + lane * (kMlpNF + 1) + f * kMlpNC;",
              "sA[t] = ra;", "av[a] = sA[(16 * a + r16) * 4 + g];",
              "sA4[t] = ra;", "av[a] = sA4[(16 * a + r16) * 4 + g];"):
        assert s in src, s
    # the inference kernel's barrier sequence around the layers
    i = src.index("mma(sf, kLdF, kMlpIn, wt.W[3], acc3, wt.W[0], acc);")
    seq = src[i:src.index("// ---- resampling to the lattice levels")]
    order = [l.strip().split("(")[0] for l in seq.splitlines()
             if l.strip().startswith(("mma(", "__syncthreads", "store_h"))]
    assert order == ["mma", "__syncthreads", "store_h", "__syncthreads", "mma", "__syncthreads", "store_h",
                     "__syncthreads", "mma", "__syncthreads", "__syncthreads"], order


class Interval:
    """Accesses of one barrier interval to one LDS array: per byte, the wave
    that wrote it; a write or read by another wave is a race."""

    def __init__(self, nbytes):
        self.n = nbytes
        self.writer = np.full(nbytes, -1, dtype=np.int32)
        self.reads = []

    def write(self, wave, off, size):
        assert 0 <= off and off + size <= self.n, (off, size, self.n)
        w = self.writer[off:off + size]
        assert np.all((w == -1) | (w == wave)), ("two waves write", off)
        w[:] = wave

    def read(self, wave, off, size):
        assert 0 <= off and off + size <= self.n, (off, size, self.n)
        self.reads.append((wave, off, size))

    def check(self):
        for wave, off, size in self.reads:
            w = self.writer[off:off + size]
            assert np.all((w == -1) | (w == wave)), ("read of another wave's write", off)


def lanes(nwaves):
    for wave in range(nwaves):
        for lane in range(64):
            yield wave, lane, lane % 16, lane // 16


def mma_reads(iv, ld, K):
    K32 = K & ~31
    for wave, lane, r16, g in lanes(NWV):
        for a in range(4):
            for k in range(0, K32, 32):
                iv.read(wave, ((16 * a + r16) * ld + k + 8 * g) * 2, 16)
            if K > K32:
                iv.read(wave, ((16 * a + r16) * ld + K32 + 4 * g) * 2, 8)


def store_h(iv):
    for wave, lane, r16, g in lanes(NWV):
        for a in range(4):
            for c in range(2):
                for i in range(4):
                    row, cl = 16 * a + 4 * g + i, 32 * wave + 16 * c + r16
                    iv.write(wave, (row * LDH + cl) * 2, 2)


def test_inference_kernel_intervals_race_free():
    ivs = []
    # features: lane = row (column of the mesh), wave q = canonical levels q, q + 8, ...
    iv = Interval(REG)
    for q, lane, _, _ in lanes(NWV):
        for c in range(q, NC, NWV):
            for f in range(3):
                iv.write(q, (lane * LDF + f * NC + c) * 2, 2)
        if q == 0:
            for i in range(NF, IN):
                iv.write(q, (lane * LDF + i) * 2, 2)
    ivs.append(iv)
    # every feature the layer-1 pass reads was written
    assert np.all(iv.writer[:64 * LDF * 2].reshape(64, LDF * 2)[:, :IN * 2] >= 0)
    iv = Interval(REG); mma_reads(iv, LDF, IN); ivs.append(iv)       # layer 1 and bypass
    iv = Interval(REG); store_h(iv); ivs.append(iv)                   # H1
    iv = Interval(REG); mma_reads(iv, LDH, HID); ivs.append(iv)       # layer 2
    iv = Interval(REG); store_h(iv); ivs.append(iv)                   # H2
    iv = Interval(REG); mma_reads(iv, LDH, HID); ivs.append(iv)       # layer 3
    iv = Interval(REG)                                                # outputs
    for wave, lane, r16, g in lanes(NWV):
        for a in range(4):
            for c in range(2):
                for i in range(4):
                    row, cl = 16 * a + 4 * g + i, 32 * wave + 16 * c + r16
                    if cl < NF:
                        iv.write(wave, (row * (NF + 1) + cl) * 4, 4)
    ivs.append(iv)
    iv = Interval(REG)                                                # resampling: lo, lo + 1 of any interval
    for wave, lane, _, _ in lanes(NWV):
        for f in range(3):
            for lo in range(NC - 1):
                iv.read(wave, (lane * (NF + 1) + f * NC + lo) * 4, 8)
    ivs.append(iv)
    for iv in ivs:
        iv.check()


def test_gemm_kernel_slices_race_free():
    # 256 threads: each slice is written (thread t: octet t % 4 of row t / 4)
    # between one pair of barriers and read between the next
    for unit in (16, 8):   # half8 slices, then the half4 remainder
        w = Interval(64 * 4 * 16)
        for t in range(256):
            w.write(t // 64, t * unit, unit)
        r = Interval(64 * 4 * 16)
        for wave, lane, r16, g in lanes(4):
            for a in range(4):
                r.read(wave, ((16 * a + r16) * 4 + g) * unit, unit)
        w.check(); r.check()
        assert np.all(w.writer[:256 * unit] >= 0)


def test_replay_finds_a_missing_barrier():
    """The checker is not vacuous: with the barrier between the H1 writes and
    the layer-2 reads taken out (one interval for both), or the one between
    the layer-1 reads and the H1 writes, it reports a race."""
    import pytest
    iv = Interval(REG)
    store_h(iv)
    mma_reads(iv, LDH, HID)
    with pytest.raises(AssertionError):
        iv.check()
    iv = Interval(REG)
    mma_reads(iv, LDF, IN)
    store_h(iv)
    with pytest.raises(AssertionError):
        # reads recorded first: check them against the writes after them
        iv.check()
