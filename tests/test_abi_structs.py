"""The ctypes mirrors of the C ABI's structures (paper_1608_06577_amd/kt.py)
against their declarations in include/kt.h: the same fields, in the same
order, with the same types and array lengths, so that a field added to one
side only fails here rather than shifting every later field at run time."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

C_TYPES = {"int32_t": C.c_int32, "int64_t": C.c_int64, "double": C.c_double}


def c_structs():
    """name -> [(field, ctype)] for every `typedef struct { ... } name;` of kt.h."""
    src = open(os.path.join(ROOT, "include", "kt.h")).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct\s*\{(.*?)\}\s*(\w+)\s*;", src, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = " ".join(decl.split())
            if not decl:
                continue
            m = re.match(r"(const )?(\w+)\s*(\*?)\s*(.*)", decl)
            base, ptr, names = m.group(2), m.group(3), m.group(4)
            for item in names.split(","):
                item = item.strip()
                star = ptr or item.startswith("*")
                item = item.lstrip("*").strip()
                # a pointer declarator may carry "const" after the star
                item = re.sub(r"^const\s+", "", item)
                mm = re.match(r"(\w+)(?:\[(\w+)\])?$", item)
                assert mm, (name, decl)
                ctype = C.c_void_p if star else C_TYPES[base]
                n = mm.group(2)
                if n is not None:
                    ctype = ctype * int(n)
                fields.append((mm.group(1), ctype))
        out[name] = fields
    return out


def same_type(a, b):
    if hasattr(a, "_length_") or hasattr(b, "_length_"):
        return (getattr(a, "_length_", None) == getattr(b, "_length_", None)
                and same_type(a._type_, b._type_))
    return a is b or (issubclass(a, C._Pointer) and b is C.c_void_p) or (
        issubclass(b, C._Pointer) and a is C.c_void_p)


@pytest.mark.parametrize("cname,pyname", [("kt_eos", "KtEos"), ("kt_params", "KtParams"),
                                           ("kt_init_state", "KtInitState"), ("kt_fields", "KtFields"),
                                           ("kt_obs", "KtObs"), ("kt_profile", "KtProfile")])
def test_struct_mirrors_match_the_header(cname, pyname):
    from paper_1608_06577_amd import kt
    decl = c_structs()[cname]
    mirror = getattr(kt, pyname)._fields_
    assert [f for f, _ in decl] == [f for f, _ in mirror], cname
    for (f, a), (_, b) in zip(decl, mirror):
        assert same_type(a, b), (cname, f, a, b)
