"""CPU test of the binding's teardown order: servers, then batches, then
contexts still open at exit are closed by the exit hook while torch is
alive; closing a context first closes the servers and batches made on it;
destructors do nothing during interpreter finalisation (where a library
call could reach a torn-down torch allocator)."""
import paper_2303_14335_amd as mp


class _FakeLib:
    def __init__(self):
        self.calls = []

    def mpld_server_destroy(self, h):
        self.calls.append(("server", h.value))

    def mpld_batch_free(self, h):
        self.calls.append(("batch", h.value))

    def mpld_context_destroy(self, h):
        self.calls.append(("context", h.value))


def _fake(cls, value):
    import ctypes
    obj = object.__new__(cls)
    obj.handle = ctypes.c_void_p(value)
    mp._register(obj)
    return obj


def test_exit_hook_closes_servers_then_batches_then_contexts(monkeypatch):
    fake = _FakeLib()
    monkeypatch.setattr(mp, "_lib", fake)
    c = _fake(mp.Context, 1)
    b = _fake(mp.Batch, 2)
    s = _fake(mp.Server, 3)
    mp._close_all()
    kinds = [k for k, _ in fake.calls]
    assert kinds == ["server", "batch", "context"], fake.calls
    # closed objects are not closed again
    mp._close_all()
    assert len(fake.calls) == 3
    del c, b, s


def test_destructor_is_inert_during_finalisation(monkeypatch):
    fake = _FakeLib()
    monkeypatch.setattr(mp, "_lib", fake)
    monkeypatch.setattr(mp, "_finalizing", lambda: True)
    c = _fake(mp.Context, 7)
    c.__del__()
    assert fake.calls == []
    monkeypatch.setattr(mp, "_finalizing", lambda: False)
    c.__del__()
    assert fake.calls == [("context", 7)]


def _fake_on(cls, value, ctx):
    import ctypes
    obj = object.__new__(cls)
    obj.handle = ctypes.c_void_p(value)
    obj.ctx = ctx
    mp._register(obj)
    return obj


def test_context_close_closes_its_servers_and_batches_first(monkeypatch):
    fake = _FakeLib()
    monkeypatch.setattr(mp, "_lib", fake)
    c = _fake(mp.Context, 11)
    other = _fake(mp.Context, 12)
    b = _fake_on(mp.Batch, 13, c)
    s = _fake_on(mp.Server, 14, c)
    kept = _fake_on(mp.Server, 15, other)
    c.close()
    assert fake.calls == [("server", 14), ("batch", 13), ("context", 11)], fake.calls
    mp._close_all()   # only the other context's objects are left
    assert fake.calls[3:] == [("server", 15), ("context", 12)], fake.calls
    del c, other, b, s, kept


def test_del_after_module_globals_cleared(monkeypatch):
    """At exit the module's globals can be cleared before the last objects
    are collected; their destructors must then do nothing, quietly."""
    fake = _FakeLib()
    monkeypatch.setattr(mp, "_lib", fake)
    c = _fake(mp.Context, 21)
    b = _fake_on(mp.Batch, 22, c)
    monkeypatch.setattr(mp, "_finalizing", None)
    b.__del__()
    c.__del__()
    assert fake.calls == []
    monkeypatch.setattr(mp, "_finalizing", lambda: False)
    c.close()
    assert fake.calls == [("batch", 22), ("context", 21)]
