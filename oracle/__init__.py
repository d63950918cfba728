"""Oracle package (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` import anything from here. The product library and its Python
binding never do.
"""
