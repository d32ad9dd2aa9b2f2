"""Register and scratch budgets of the built gfx950 kernels, read from the
AMDGPU metadata note of every code object in libstf.so (no GPU needed).

The forward kernels are register-budgeted per texture count: the whole-tile
kernels issue VALU most of the time and hide their memory and LDS latency
with resident waves (waves per SIMD = 512 / the VGPR budget). Per-lane data kept
in scratch memory costs memory traffic on every wave; a runtime-indexed
copy of the per-slot picks once kept all of them in scratch in the
four-texture whole-tile kernel and made it 1.6x slower."""
import re
import struct

import msgpack
import pytest

import paper_2504_05562_amd as stf

MODES = {0: "stf", 1: "quad", 2: "records", 3: "bins"}
BUNDLE_MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"
NT_AMDGPU_METADATA = 32


def _sections(elf):
    """(name, type, offset, size) of every section of an ELF64 image."""
    shoff, = struct.unpack_from("<Q", elf, 0x28)
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", elf, 0x3A)
    hdrs = [struct.unpack_from("<IIQQQQIIQQ", elf, shoff + i * shentsize) for i in range(shnum)]
    strtab = hdrs[shstrndx][4]
    out = []
    for h in hdrs:
        start = strtab + h[0]
        out.append((elf[start:elf.index(b"\0", start)].decode(), h[1], h[4], h[5]))
    return out


def _code_objects(lib):
    """The gfx950 code objects of the offload bundles in .hip_fatbin."""
    fatbin = [lib[o:o + s] for name, _, o, s in _sections(lib) if name == ".hip_fatbin"]
    assert len(fatbin) == 1, "libstf.so has no .hip_fatbin section"
    fb = fatbin[0]
    for m in re.finditer(re.escape(BUNDLE_MAGIC), fb):
        base = m.start()
        n, = struct.unpack_from("<Q", fb, base + len(BUNDLE_MAGIC))
        p = base + len(BUNDLE_MAGIC) + 8
        for _ in range(n):
            off, size, tlen = struct.unpack_from("<QQQ", fb, p)
            p += 24
            triple = fb[p:p + tlen].decode()
            p += tlen
            if triple.endswith("gfx950"):
                yield fb[base + off:base + off + size]


def _kernels(co):
    for _, typ, off, size in _sections(co):
        if typ != 7:                                   # SHT_NOTE
            continue
        q = off
        while q < off + size:
            nsz, dsz, ntype = struct.unpack_from("<III", co, q)
            q += 12 + ((nsz + 3) & ~3)
            desc = co[q:q + dsz]
            q += (dsz + 3) & ~3
            if ntype == NT_AMDGPU_METADATA:
                yield from msgpack.unpackb(desc, raw=False)["amdhsa.kernels"]


@pytest.fixture(scope="module")
def kernels():
    with open(stf.lib_path, "rb") as f:
        lib = f.read()
    out = {}
    for co in _code_objects(lib):
        for k in _kernels(co):
            out[k[".name"]] = k
    assert out, "no kernel metadata found"
    return out


def _forward(kernels):
    """{(filter, mode, textures, decoder, exact): metadata} of forward_kernel."""
    pat = re.compile(r"forward_kernelILi(\d)ELi(\d)ELi(\d)ELb([01])ELb([01])E")
    out = {}
    for name, k in kernels.items():
        m = pat.search(name)
        if m:
            filt, mode, nt, dec, ef = (int(g) for g in m.groups())
            out[(filt, MODES[mode], nt, bool(dec), bool(ef))] = k
    return out


def test_every_forward_instantiation_is_present(kernels):
    fwd = _forward(kernels)
    for filt in (0, 1):
        for mode in MODES.values():
            for nt in (1, 2, 3, 4):
                for dec in (False, True):
                    # exact filtering (coverage) exists for the reuse modes only
                    for ef in ((False,) if mode == "stf" else (False, True)):
                        assert (filt, mode, nt, dec, ef) in fwd, (filt, mode, nt, dec, ef)
    assert len(fwd) == 2 * 4 * (2 + 3 * 4)
    assert any("backward_kernel" in n for n in kernels)
    assert any("estimator_kernel" in n for n in kernels)
    assert any("reference_kernel" in n for n in kernels)


@pytest.mark.parametrize("filt", [0, 1], ids=["bilinear", "bicubic"])
def test_whole_tile_kernels_keep_their_register_budget(kernels, filt):
    fwd = _forward(kernels)
    for nt, budget in ((1, 64), (2, 64), (3, 72), (4, 80)):
        k = fwd[(filt, "bins", nt, False, False)]
        assert k[".vgpr_count"] + k[".agpr_count"] <= budget, (nt, k[".vgpr_count"])
    for nt in (1, 2, 3, 4):                              # latent decoder: four waves
        k = fwd[(filt, "bins", nt, True, False)]
        assert k[".vgpr_count"] + k[".agpr_count"] <= 128, (nt, k[".vgpr_count"])


@pytest.mark.parametrize("filt", [0, 1], ids=["bilinear", "bicubic"])
def test_forward_kernels_keep_per_lane_data_in_registers(kernels, filt):
    fwd = _forward(kernels)
    for mode in MODES.values():
        for nt in (1, 2, 3, 4):
            k = fwd[(filt, mode, nt, False, False)]
            # the whole-tile kernel spills a few registers with two textures at
            # 64 VGPRs and with four at 80
            limit = {2: 32, 4: 64}.get(nt, 0) if mode == "bins" else 0
            assert k[".private_segment_fixed_size"] <= limit, (mode, nt, k[".private_segment_fixed_size"])
            assert not k[".uses_dynamic_stack"], (mode, nt)
    # the one-texture latent whole-tile kernel spills a few registers at its 128-VGPR budget
    assert fwd[(filt, "bins", 1, True, False)][".private_segment_fixed_size"] <= 32
    # with several latent textures the exchanging decoder kernels run their slots one after
    # another (spilling some registers at 128 VGPRs) instead of keeping every slot's pick in
    # scratch memory, which took 336-432 bytes per lane
    for mode in ("quad", "records", "bins"):
        for nt in (2, 3, 4):
            k = fwd[(filt, mode, nt, True, False)]
            assert k[".private_segment_fixed_size"] <= 256, (mode, nt, k[".private_segment_fixed_size"])
    # exact filtering with three or four textures runs its slots one after another: no scratch
    for mode in ("quad", "records", "bins"):
        for nt in (3, 4):
            assert fwd[(filt, mode, nt, False, True)][".private_segment_fixed_size"] == 0, (mode, nt)


def test_other_kernels_use_no_scratch(kernels):
    for name, k in kernels.items():
        # forward kernels: above; the latent Eq. (3) kernel (16 decodes per pixel) is not budgeted
        if "forward_kernel" in name or re.search(r"reference_kernelILi\dELb1E", name):
            continue
        # the bicubic exchange adjoints spill a few registers at their budgets (96 VGPRs, 128 for the records)
        limit = 32 if re.fullmatch(r"_ZN3stf15backward_kernelILi1ELi[123]EEEvNS_4ArgsE", name) else 0
        assert k[".private_segment_fixed_size"] <= limit, name
        assert not k[".uses_dynamic_stack"], name


def test_adjoint_occupancy(kernels):
    """Five waves per SIMD (96 VGPRs, five workgroups' LDS per CU); the
    record footprints' adjoint four (128 VGPRs)."""
    for filt in (0, 1):
        for mode in range(4):
            waves = 4 if mode == 2 else 5
            k = kernels["_ZN3stf15backward_kernelILi%dELi%dEEEvNS_4ArgsE" % (filt, mode)]
            assert k[".vgpr_count"] + k[".agpr_count"] <= 512 // waves // 8 * 8, (filt, mode)
            assert k[".group_segment_fixed_size"] * waves <= 160 * 1024, (filt, mode)


def test_shared_records_kernel_keeps_eight_waves(kernels):
    """The one-size shared-selection record kernel (two or three textures)
    fits 64 VGPRs without scratch, so it holds eight waves per SIMD."""
    for filt in (0, 1):
        for nt in (2, 3):
            k = kernels["_ZN3stf21shared_records_kernelILi%dELi%dEEEvNS_4ArgsE" % (filt, nt)]
            assert k[".vgpr_count"] + k[".agpr_count"] <= 64, (filt, nt)
            assert k[".private_segment_fixed_size"] == 0, (filt, nt)
