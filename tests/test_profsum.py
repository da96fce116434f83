"""The profile summaries' kernel-name table: every chunked-pass kernel that the
kernel translation unit launches, instantiated the way rocprofv3 prints it,
maps to the profiling slot of its pass (the slots the traffic summaries and
the bench's live timings share)."""
import os
import re

import pytest

import profsum

HERE = os.path.dirname(os.path.abspath(__file__))
KERN = os.path.join(HERE, "..", "paper_1902_10078_amd", "csrc", "bandops_kern.hip")

# template name and its boolean arguments -> slot
EXPECTED = {
    ("k_f1_sum", ("false",)): "f1_summary",
    ("k_f1_sum", ("true",)): "f1_summary",
    ("k_f1_sum_q", ("false",)): "f1_summary",
    ("k_f1_sum_q", ("true",)): "f1_summary",
    ("k_f1_rep", ("false", "false")): "f1_replay",
    ("k_f1_rep", ("false", "true")): "f1_replay",
    ("k_f1_rep", ("true", "false", "false")): "f1_replay",
    ("k_f1_rep", ("true", "true", "false")): "f1_replay",
    ("k_pc", ()): "chunk_product",
    ("k_fs", ("false", "false")): "fs_summary",
    ("k_fs", ("true", "false")): "fs_replay",
    ("k_fs", ("true", "true")): "fs_replay",
    ("k_f2", ("false", "false")): "f2_summary",
    ("k_f2", ("true", "false")): "f2_replay",
    ("k_f2", ("true", "true")): "f2_replay",
    ("k_b1", ("false", "false")): "b1_summary",
    ("k_b1", ("true", "false")): "b1_replay",
    ("k_b1", ("true", "true")): "b1_replay",
    ("k_b2", ("false", "false")): "b2_summary",
    ("k_b2", ("false", "true")): "b2_summary",
    ("k_b2", ("true", "false")): "b2_replay",
    ("k_b2", ("true", "true")): "b2_replay",
    ("k_f1_gscan", ()): "f1_group_compose",
    ("k_f1_gcomp_q", ()): "f1_group_compose",
    ("k_lin_gcomp_q", ("true",)): "desc_group_compose",
    ("k_lin_gcomp_q", ("false",)): "asc_group_compose",
    ("k_f1_pscan", ()): "f1_group_sweep",
    ("k_f1_sweep_q", ("true",)): "f1_group_sweep",
    ("k_f1_sweep_q", ("false",)): "f1_chunk_sweep",
    ("k_lin_sweep_q", ("true", "true")): "desc_group_sweep",
    ("k_lin_sweep_q", ("true", "false")): "desc_chunk_sweep",
    ("k_lin_sweep_q", ("false", "true")): "asc_group_sweep",
    ("k_lin_sweep_q", ("false", "false")): "asc_chunk_sweep",
    ("k_f1_capply", ()): "f1_chunk_sweep",
    ("k_lin_gscan", ("true",)): "desc_group_compose",
    ("k_lin_pscan", ("true",)): "desc_group_sweep",
    ("k_lin_capply", ("true",)): "desc_chunk_sweep",
    ("k_lin_gscan", ("false",)): "asc_group_compose",
    ("k_lin_pscan", ("false",)): "asc_group_sweep",
    ("k_lin_capply", ("false",)): "asc_chunk_sweep",
}


def launched_kernels():
    src = open(KERN).read()
    out = set()
    for m in re.finditer(r"hipLaunchKernelGGL\(\((k_\w+)<([^>]*)>\)", src):
        args = [a.strip() for a in m.group(2).split(",")]
        out.add((m.group(1), tuple(a for a in args if a in ("true", "false"))))
    return out


def printed_name(name, bools, t):
    # as rocprofv3 prints an instantiation at K = 5
    args = ["5"] + ([t] if name not in ("k_f1_gscan", "k_f1_pscan", "k_f1_capply", "k_f1_gcomp_q",
                                                  "k_f1_sweep_q") and
                    not name.startswith("k_lin_") else []) + list(bools)
    return f"void (anonymous namespace)::{name}<{', '.join(args)}>(bo::Args, long)"


def test_every_launched_kernel_is_listed():
    assert launched_kernels() == set(EXPECTED)


@pytest.mark.parametrize("t", ["double", "float"])
def test_slots_of_launched_kernels(t):
    for (name, bools), slot in EXPECTED.items():
        assert profsum.slot_of(printed_name(name, bools, t)) == slot, (name, bools, t)
