"""The batched kernels read their frames from a device table whose pointers
are stored as offsets from the table's address (the host converts them on
upload, each kernel adds the address back). Both sides take the member list
from one macro; this checks on the CPU that the macro names every pointer
member of the frame, so that no pointer reaches a kernel unconverted."""
import os
import re

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "paper_1802_07210_amd", "csrc", "elas_internal.h")


def _source():
    with open(HEADER) as f:
        return f.read()


def frame_pointer_members(src):
    body = re.search(r"struct Frame \{(.*?)\n\};", src, re.S).group(1)
    names = []
    for line in body.split("\n"):
        code = line.split("//")[0].strip()
        m = re.match(r"(?:const\s+)?[\w:]+\s*\*\s*(\w+)\s*;", code)
        if m:
            names.append(m.group(1))
    return names


def macro_members(src):
    m = re.search(r"#define ELAS_FRAME_POINTERS\(X\)((?:.*\\\n)*.*)", src)
    return re.findall(r"X\((\w+)\)", m.group(1))


def test_every_frame_pointer_is_converted():
    src = _source()
    members = frame_pointer_members(src)
    listed = macro_members(src)
    assert len(members) >= 40
    assert sorted(members) == sorted(listed)
    assert len(set(listed)) == len(listed)


def test_both_sides_use_the_list():
    src = _source()
    assert re.search(r"inline void frame_to_table\(Frame\* f, uintptr_t table\).*?"
                     r"ELAS_FRAME_POINTERS\(ELAS_TO_OFFSET\)", src, re.S)
    assert re.search(r"Frame global_frame\(const Frame& t, const char\* base\).*?"
                     r"ELAS_FRAME_POINTERS\(ELAS_FROM_OFFSET\)", src, re.S)
