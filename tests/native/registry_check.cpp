// CPU check of the context's simulation bookkeeping (fskmc_registry.h),
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_registry.py.  Simulations are heap objects as in the library,
// so a list that kept a destroyed simulation would be a use after free.
#include <cstdio>
#include <cstdlib>

#include "../../paper_1105_4673_amd/csrc/fskmc_registry.h"

struct Sim {
    int id;
    bool invalid = false;
};

#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                                 \
        }                                                                 \
    } while (0)

// What the library does after a synchronising call: the sticky flag decides
// whether every simulation touched since the last check becomes invalid.
static void settle(fskmc::SimRegistry<Sim>& r, bool flag)
{
    for (Sim* s : r.settle(flag))
        s->invalid = true;
}

int main()
{
    fskmc::SimRegistry<Sim> r;
    Sim* a = new Sim{1};
    Sim* b = new Sim{2};
    Sim* c = new Sim{3};
    r.add(a);
    r.add(b);
    r.add(c);
    CHECK(r.n_live() == 3 && r.n_pending() == 0);

    // two persistent launches before one synchronisation: the first aborted,
    // the second ran cleanly; the flag stays raised, so both sims are hit
    r.touched(a);
    r.touched(b);
    r.touched(a);  // repeated launches of one sim are recorded once
    CHECK(r.n_pending() == 2);
    settle(r, true);
    CHECK(a->invalid && b->invalid && !c->invalid);
    CHECK(r.n_pending() == 0);

    // a clean synchronisation forgets the pending list without marking
    a->invalid = b->invalid = false;
    r.touched(c);
    settle(r, false);
    CHECK(!c->invalid && r.n_pending() == 0);

    // destroying a sim with a launch pending removes it from both lists: the
    // next settle must not reach the freed object
    r.touched(b);
    r.touched(c);
    r.remove(b);
    delete b;
    CHECK(r.n_live() == 2 && r.n_pending() == 1 && !r.is_live(b));
    settle(r, true);
    CHECK(c->invalid && !a->invalid);

    // destroying the context hands over every live sim exactly once
    r.touched(a);
    std::vector<Sim*> all = r.release_all();
    CHECK(all.size() == 2 && r.n_live() == 0 && r.n_pending() == 0);
    for (Sim* s : all)
        delete s;
    settle(r, true);  // nothing left to mark
    CHECK(r.settle(false).empty());
    std::puts("registry ok");
    return 0;
}
