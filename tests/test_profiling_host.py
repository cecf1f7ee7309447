"""Host logic of the profile summaries: the source hash that decides whether a
committed counter record still describes the current kernels ignores comments
and layout but not code."""
from paper_1909_09825_amd.profiling import code_text


def test_code_text_drops_comments_keeps_literals():
    src = ('int a = 1;  // trailing\n/* block\n   comment */ const char* s = "x // y /* z */";\n'
           "char q = '/'; char e = '\\\\'; int b = a / 2;\n")
    assert code_text(src) == ('int a = 1; const char* s = "x // y /* z */"; char q = \'/\'; '
                              "char e = '\\\\'; int b = a / 2;")


def test_comment_edits_keep_the_text_code_edits_change_it():
    base = "__global__ void k(int* p) {\n  // one\n  p[0] = 1;  /* two */\n}\n"
    reworded = "__global__ void k(int* p) {\n  // a different comment\n\n  p[0] = 1;\n}\n"
    changed = "__global__ void k(int* p) {\n  // one\n  p[0] = 2;  /* two */\n}\n"
    assert code_text(base) == code_text(reworded)
    assert code_text(base) != code_text(changed)
