"""Host-side wiring: every field of the kernel argument structs that a
search launch fills is assigned at its launch site (a field left at its zero
initialiser would hand a null pointer to a kernel).  Source-level check, runs
without a GPU; the launchers also refuse null pointers at run time."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2402_13435_amd", "csrc")


def struct_fields(name):
    text = open(os.path.join(CSRC, "fr_internal.h")).read()
    body = re.search(r"struct %s \{(.*?)\n\};" % name, text, re.S).group(1)
    body = re.sub(r"//[^\n]*", "", body)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        for part in decl.split(","):
            m = re.search(r"(\w+)\s*$", part.strip())
            if m:
                fields.append(m.group(1))
    return fields


def assigned(var):
    text = open(os.path.join(CSRC, "fr_runtime.cpp")).read()
    return set(re.findall(r"\b%s\.(\w+)\s*=" % var, text))


def test_search_launch_args_fully_assigned():
    for struct, var in (("PrepArgs", "pa"), ("ScanArgs", "sa"), ("SelectArgs", "se"),
                        ("RescoreArgs", "rs"),
                        ("MaskWordArgs", "ma"), ("SeedArgs", "sd"),
                        ("RouteArgs", "ra"), ("SparseRowsArgs", "sr"), ("RowDotArgs", "rd"),
                        ("QuantArgs", "qs"), ("QuantSelectArgs", "qc")):
        missing = set(struct_fields(struct)) - assigned(var)
        assert not missing, f"{struct} {var}: unassigned {sorted(missing)}"


def test_launchers_guard_pointers():
    text = "".join(open(os.path.join(CSRC, f)).read()
                   for f in ("fr_kernels.hip", "fr_quant.hip", "fr_sparse.hip"))
    # pointers a launcher may receive as null (the kernel then does not read
    # them), each guarded conditionally or documented as optional
    for launcher, struct, optional in (
            ("launch_prep", "PrepArgs", set()), ("launch_scan", "ScanArgs", {"xscale", "qscale"}),
            ("launch_select", "SelectArgs", set()),
            ("launch_rescore", "RescoreArgs", set()),
            ("launch_mask_words", "MaskWordArgs", {"run_if"}),
            ("launch_seed", "SeedArgs", {"xscale", "qscale"}),
            ("launch_route", "RouteArgs", {"kp"}),
            ("launch_sparse_rows", "SparseRowsArgs", set()),
            ("launch_row_dots", "RowDotArgs", {"qlist", "n_list", "master", "tiles", "hist"}),
            ("launch_sign_codes", "SignArgs", {"n_dev", "slots"}),
            ("launch_quant_cut", "QuantSelectArgs", {"ties", "surv", "slot_ids"}),
            ("launch_quant_ties", "QuantSelectArgs", {"k", "hist", "thr", "tau", "hinvw",
                                                      "tsafe", "ovf"})):
        body = text[text.index("hipError_t %s(" % launcher):]
        body = body[:body.index("\n}\n")]
        guarded = set(re.findall(r"FR_REQUIRE\(a\.(\w+)\)", body))
        hdr = open(os.path.join(CSRC, "fr_internal.h")).read()
        sbody = re.search(r"struct %s \{(.*?)\n\};" % struct, hdr, re.S).group(1)
        ptrs = set(re.findall(r"\*\s*(\w+)\s*;", re.sub(r"//[^\n]*", "", sbody)))
        assert ptrs - guarded - optional == set(), (launcher, sorted(ptrs - guarded - optional))
